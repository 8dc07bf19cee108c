// Host number theory, double-double canonical-embedding codec, sampler.
//
// The encoder evaluates tau^{-1} (Cheon-Kim-Kim-Song 2017) as an inverse DFT
// of size N over the primitive 2N-th roots, in double-double arithmetic
// (Dekker two-sum/two-product; Bailey's QD formulas), with twiddles from a
// Taylor series in double-double, so the value that is rounded to an integer
// carries ~100 correct bits and the rounding matches the exact value except
// on a vanishing set of inputs.  Compiled with -ffp-contract=off.
#include "host_math.h"

#include <cmath>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>

namespace fh {

u64 powmod(u64 a, u64 e, u64 q) {
  u64 r = 1 % q;
  a %= q;
  for (; e; e >>= 1) {
    if (e & 1) r = mulmod(r, a, q);
    a = mulmod(a, a, q);
  }
  return r;
}

u64 invmod(u64 a, u64 q) {
  if (a % q == 0) throw std::runtime_error("invmod of zero");
  return powmod(a, q - 2, q);
}

// Deterministic Miller-Rabin for 64-bit integers with the seven bases of
// Jaeschke / Sinclair.
bool prime64(u64 n) {
  if (n < 2) return false;
  for (u64 p : {2ull, 3ull, 5ull, 7ull, 11ull, 13ull}) {
    if (n % p == 0) return n == p;
  }
  u64 d = n - 1;
  int r = 0;
  while (!(d & 1)) { d >>= 1; r++; }
  for (u64 a : {2ull, 325ull, 9375ull, 28178ull, 450775ull, 9780504ull, 1795265022ull}) {
    u64 b = a % n;
    if (b == 0) continue;
    u64 x = powmod(b, d, n);
    if (x == 1 || x == n - 1) continue;
    bool witness = true;
    for (int i = 1; i < r && witness; i++) {
      x = mulmod(x, x, n);
      if (x == n - 1) witness = false;
    }
    if (witness) return false;
  }
  return true;
}

std::vector<u64> ntt_primes(int bits, int logn, int count, const std::vector<u64>& skip) {
  const u64 step = 2ull << logn;
  std::vector<u64> out;
  for (u64 p = ((1ull << bits) - 2) / step * step + 1; (int)out.size() < count; p -= step) {
    if (p < step) throw std::runtime_error("not enough NTT-friendly primes");
    bool skipped = false;
    for (u64 s : skip) skipped |= (s == p);
    if (!skipped && prime64(p)) out.push_back(p);
  }
  return out;
}

u64 root_2n(u64 p, int logn) {
  const u64 twoN = 2ull << logn;
  for (u64 x = 2;; x++) {
    u64 r = powmod(x, (p - 1) / twoN, p);
    if (powmod(r, twoN / 2, p) == p - 1) return r;
  }
}

unsigned bitrev(unsigned x, int bits) {
  unsigned r = 0;
  for (int i = 0; i < bits; i++, x >>= 1) r = (r << 1) | (x & 1);
  return r;
}

// ------------------------------------------------------------------ sampler
u64 splitmix_mix(u64 z) {
  z ^= z >> 30;
  z *= 0xbf58476d1ce4e5b9ull;
  z ^= z >> 27;
  z *= 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

u64 stream_word(u64 seed, u64 tag, u64 i) {
  u64 state = splitmix_mix(seed ^ (tag * 0xD1B54A32D192ED03ull));
  state += (i + 1) * 0x9E3779B97F4A7C15ull;
  return splitmix_mix(state);
}

int draw_ternary(u64 seed, u64 tag, u64 i) {
  return (int)(((u128)stream_word(seed, tag, i) * 3u) >> 64) - 1;
}

u64 draw_uniform(u64 seed, u64 tag, u64 i, u64 q) {
  const u128 v = ((u128)stream_word(seed, tag, 2 * i) << 64) | stream_word(seed, tag, 2 * i + 1);
  return (u64)(v % q);
}

// ------------------------------------------------------------------ double-double
namespace {

struct dd {
  double hi, lo;
};

inline dd two_sum(double a, double b) {
  double s = a + b, bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
inline dd quick(double a, double b) {
  double s = a + b;
  return {s, b - (s - a)};
}
inline dd add(dd x, dd y) {
  dd s = two_sum(x.hi, y.hi), t = two_sum(x.lo, y.lo);
  s.lo += t.hi;
  s = quick(s.hi, s.lo);
  s.lo += t.lo;
  return quick(s.hi, s.lo);
}
inline dd neg(dd x) { return {-x.hi, -x.lo}; }
inline dd sub(dd x, dd y) { return add(x, neg(y)); }
inline dd mul(dd x, dd y) {
  double p = x.hi * y.hi, e = std::fma(x.hi, y.hi, -p);
  e += x.hi * y.lo;
  e += x.lo * y.hi;
  return quick(p, e);
}
inline dd mul_d(dd x, double d) {
  double p = x.hi * d, e = std::fma(x.hi, d, -p);
  e += x.lo * d;
  return quick(p, e);
}
inline dd div(dd x, dd y) {
  double q1 = x.hi / y.hi;
  dd r = sub(x, mul(y, {q1, 0}));
  double q2 = r.hi / y.hi;
  r = sub(r, mul(y, {q2, 0}));
  double q3 = r.hi / y.hi;
  return add(quick(q1, q2), {q3, 0});
}

const dd kTwoPi = {6.283185307179586232, 2.4492935982947064e-16};

struct Tables {
  std::vector<dd> wc, ws;   // e^{2 pi i k / N},  k < N/2
  std::vector<dd> zc, zs;   // e^{pi i k / N},    k < N
};

dd div_int(dd x, double d) {
  return div(x, {d, 0});
}

// cos and sin of 2*pi*k/M (M a power of two): octant reduction, then the
// Taylor series in double-double with exact division of each term
void cis_exact(long long k, long long M, dd& c, dd& s) {
  k %= M;
  if (k < 0) k += M;
  bool flip_half = false, quarter = false, mirror = false;
  if (2 * k >= M) { k -= M / 2; flip_half = true; }
  if (4 * k >= M) { k -= M / 4; quarter = true; }
  if (8 * k > M) { k = M / 4 - k; mirror = true; }
  const dd th = mul_d(kTwoPi, (double)k / (double)M);
  const dd th2 = mul(th, th);
  dd cs = {1, 0}, sn = th, tc = {1, 0}, ts = th;
  for (int n = 1; n < 40; n++) {
    tc = div_int(neg(mul(tc, th2)), (2.0 * n - 1) * (2.0 * n));
    ts = div_int(neg(mul(ts, th2)), (2.0 * n) * (2.0 * n + 1));
    cs = add(cs, tc);
    sn = add(sn, ts);
    if (std::fabs(tc.hi) < 1e-36 && std::fabs(ts.hi) < 1e-36) break;
  }
  if (mirror) std::swap(cs, sn);
  if (quarter) {
    dd t = cs;
    cs = neg(sn);
    sn = t;
  }
  if (flip_half) { cs = neg(cs); sn = neg(sn); }
  c = cs;
  s = sn;
}

const Tables& tables(int logn) {
  static std::mutex mu;
  static std::map<int, std::unique_ptr<Tables>> cache;
  std::lock_guard<std::mutex> g(mu);
  auto it = cache.find(logn);
  if (it != cache.end()) return *it->second;
  auto T = std::make_unique<Tables>();
  const long long N = 1LL << logn;
  T->wc.resize(N / 2); T->ws.resize(N / 2);
  for (long long k = 0; k < N / 2; k++) cis_exact(k, N, T->wc[k], T->ws[k]);
  T->zc.resize(N); T->zs.resize(N);
  for (long long k = 0; k < N; k++) cis_exact(k, 2 * N, T->zc[k], T->zs[k]);
  const Tables& ref = *T;
  cache[logn] = std::move(T);
  return ref;
}

// in-place radix-2 DFT: X_i = sum_t x_t e^{sign 2 pi i t i / N}
void fft(std::vector<dd>& re, std::vector<dd>& im, int logn, int sign, const Tables& T) {
  const long long N = 1LL << logn;
  for (long long i = 0; i < N; i++) {
    long long j = bitrev((unsigned)i, logn);
    if (i < j) { std::swap(re[i], re[j]); std::swap(im[i], im[j]); }
  }
  for (long long len = 2; len <= N; len <<= 1) {
    const long long half = len / 2, step = N / len;
    for (long long b = 0; b < N; b += len)
      for (long long k = 0; k < half; k++) {
        const dd wr = T.wc[k * step], wi = sign > 0 ? T.ws[k * step] : neg(T.ws[k * step]);
        const long long u = b + k, v = b + k + half;
        const dd xr = sub(mul(re[v], wr), mul(im[v], wi));
        const dd xi = add(mul(re[v], wi), mul(im[v], wr));
        re[v] = sub(re[u], xr); im[v] = sub(im[u], xi);
        re[u] = add(re[u], xr); im[u] = add(im[u], xi);
      }
  }
}

int64_t round_away(dd v) {
  const bool negv = v.hi < 0 || (v.hi == 0 && v.lo < 0);
  dd a = negv ? neg(v) : v;
  a = add(a, {0.5, 0});
  double f = std::floor(a.hi);
  long double r;
  if (f == a.hi) r = (long double)f + (long double)std::floor(a.lo);
  else r = f;
  if (r > 4.6e18) throw std::runtime_error("encode: coefficient out of range");
  const int64_t m = (int64_t)r;
  return negv ? -m : m;
}

dd exp_dd(double x) {   // |x| < 32
  const dd y = {std::ldexp(x, -10), 0};
  dd s = {1, 0}, t = {1, 0};
  for (int n = 1; n < 30; n++) {
    t = div_int(mul(t, y), (double)n);
    s = add(s, t);
  }
  for (int i = 0; i < 10; i++) s = mul(s, s);
  return s;
}

}  // namespace

const std::vector<u64>& gauss_thresholds() {
  static std::vector<u64> T;
  static std::once_flag once;
  std::call_once(once, [] {
    // rho(k) = exp(-k^2 / (2 sigma^2)), sigma = 3.2 -> k^2/(2 sigma^2) = 25 k^2 / 512 exactly
    dd rho[20];
    for (int k = 0; k < 20; k++) rho[k] = exp_dd(-25.0 * k * k / 512.0);
    dd Z = rho[0];
    for (int k = 1; k < 20; k++) Z = add(Z, mul_d(rho[k], 2.0));
    dd cum = rho[0];
    for (int k = 1; k < 20; k++) {
      dd v = mul_d(div(cum, Z), 9223372036854775808.0);   // * 2^63
      double f = std::floor(v.hi);
      long double r = (f == v.hi) ? (long double)f + std::floor(v.lo) : (long double)f;
      T.push_back((u64)r);
      cum = add(cum, mul_d(rho[k], 2.0));
    }
  });
  return T;
}

int draw_gauss(u64 seed, u64 tag, u64 i) {
  const std::vector<u64>& T = gauss_thresholds();
  const u64 r = stream_word(seed, tag, i);
  const u64 u = r & 0x7FFFFFFFFFFFFFFFull;
  int mag = 0;
  for (u64 t : T) mag += (u >= t);
  return (r >> 63) ? -mag : mag;
}

void encode_real(int logn, const double* z, double scale, int64_t* m) {
  const Tables& T = tables(logn);
  const long long N = 1LL << logn, twoN = 2 * N, ns = N / 2;
  std::vector<dd> re(N, dd{0, 0}), im(N, dd{0, 0});
  long long e = 1;
  for (long long j = 0; j < ns; j++) {
    re[(e - 1) / 2] = {z[j], 0};
    re[(twoN - e - 1) / 2] = {z[j], 0};
    e = e * 5 % twoN;
  }
  fft(re, im, logn, -1, T);
  const double sN = std::ldexp(1.0, -logn);
  for (long long i = 0; i < N; i++) {
    // Re(F_i * zeta^{-i}) = Fr cos + Fi sin
    dd v = add(mul(re[i], T.zc[i]), mul(im[i], T.zs[i]));
    v = mul_d(mul_d(v, scale), sN);
    m[i] = round_away(v);
  }
}

void decode_real(int logn, const int64_t* m, double scale, double* z) {
  const Tables& T = tables(logn);
  const long long N = 1LL << logn, twoN = 2 * N, ns = N / 2;
  std::vector<dd> re(N), im(N);
  for (long long i = 0; i < N; i++) {
    const dd mi = {(double)m[i], (double)(m[i] - (int64_t)(double)m[i])};
    re[i] = mul(mi, T.zc[i]);
    im[i] = mul(mi, T.zs[i]);
  }
  fft(re, im, logn, +1, T);
  long long e = 1;
  for (long long j = 0; j < ns; j++) {
    const dd v = re[(e - 1) / 2];
    z[j] = (v.hi + v.lo) / scale;
    e = e * 5 % twoN;
  }
}

}  // namespace fh
