// Exhaustive-edge and random check of the library's binary64 modular
// arithmetic (fenc_arith.h) and of the NTT register rounds (fenc_kernels.h)
// against unsigned/signed 128-bit integer arithmetic.  Built with g++ by
// tests/test_arith.py; prints one line per check and "FAIL ..." lines for
// every violated property; exit status 1 on any failure.
//
// Properties checked (q an NTT prime of 30, 40 or 50 bits):
//   mulmod(a, b):    r = a*b - e*q exactly, r an integer, |r| < q, whenever
//                    |a*b/q| < 2^51
//   mulmod_c(a, w):  with wq = fl(w/q) or fl(w*fl(1/q)): r exact and integer
//                    whenever a*w/q > -2^51 and |a| < 2^52; |r| <= (1/2 +
//                    |a|/(4q)) q below 2^51 and (1 + |a|/(4q)) q above
//   the precondition is tight: below -2^51 some products are not integers
//   red(x):          r = x - e*q exact, |r| <= q/2 + 1, for |x| < 2^52
//   u2d / d2u:       exact round trip on [0, 2^52)
//   fwd_round<3|4> and inv_round<3|4>: outputs congruent to the exact
//                    butterfly network, |out| <= q/2 + 1 (forward) and < q
//                    (inverse), on adversarial and random inputs/twiddles
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "fenc_kernels.h"

using fk::d2;
typedef __int128 i128;
typedef unsigned __int128 u128;

static int failures = 0;
static void fail(const char* what, double a, double b, double q, double r) {
  if (failures < 40) std::printf("FAIL %s a=%.17g b=%.17g q=%.17g r=%.17g\n", what, a, b, q, r);
  failures++;
}

static uint64_t mulmod64(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }
static uint64_t powmod64(uint64_t a, uint64_t e, uint64_t m) {
  uint64_t r = 1;
  a %= m;
  while (e) {
    if (e & 1) r = mulmod64(r, a, m);
    a = mulmod64(a, a, m);
    e >>= 1;
  }
  return r;
}
// deterministic Miller-Rabin for 64-bit integers (witnesses of Jaeschke / Sinclair)
static bool is_prime(uint64_t n) {
  if (n < 2) return false;
  for (uint64_t p : {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37})
    if (n % p == 0) return n == p;
  uint64_t d = n - 1;
  int s = 0;
  while (!(d & 1)) { d >>= 1; s++; }
  for (uint64_t a : {2, 325, 9375, 28178, 450775, 9780504, 1795265022}) {
    uint64_t x = powmod64(a % n, d, n);
    if (a % n == 0 || x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int i = 1; i < s && comp; i++) {
      x = mulmod64(x, x, n);
      if (x == n - 1) comp = false;
    }
    if (comp) return false;
  }
  return true;
}
static uint64_t prime_below(int bits, int logn2) {
  const uint64_t step = 1ull << logn2;
  for (uint64_t q = ((1ull << bits) / step) * step + 1;; q -= step)
    if (q < (1ull << bits) && is_prime(q)) return q;
}

static bool is_int(double x) { return std::isfinite(x) && std::floor(x) == x && std::fabs(x) < 9007199254740992.0; }
// (x - a*b) divisible by q, all exact integers
static bool congruent_prod(double r, double a, double b, double q) {
  const i128 d = (i128)(int64_t)r - (i128)(int64_t)a * (i128)(int64_t)b;
  return d % (i128)(int64_t)q == 0;
}
static i128 emod(i128 x, i128 q) {
  i128 r = x % q;
  return r < 0 ? r + q : r;
}

static void check_mulmod(double q, std::mt19937_64& g) {
  const double qi = 1.0 / q, lim = std::ldexp(1.0, 51);
  long n = 0;
  auto one = [&](double a, double b) {
    if (!(std::fabs(a * b / q) < lim * (1 - 1e-12))) return;
    const double r = fk::mulmod(a, b, q, qi);
    n++;
    if (!is_int(r) || !congruent_prod(r, a, b, q) || !(std::fabs(r) < q)) fail("mulmod", a, b, q, r);
  };
  std::vector<double> edge = {0, 1, -1, q - 1, -(q - 1), std::floor(q / 2), -std::floor(q / 2), 2 * q - 1, -(2 * q - 1),
                              3 * q - 1, -(3 * q - 1)};
  for (double a : edge)
    for (double b : edge) one(a, b);
  // a at the edge of the band |a b / q| < 2^51 for b near +-q
  for (double b : {q - 1, -(q - 1), q - 2, std::floor(q * 0.75)})
    for (int k = 0; k < 64; k++) {
      const double a = std::floor(lim * q / std::fabs(b) * (1 - 1e-9)) - k;
      one(a, b);
      one(-a, b);
    }
  std::uniform_real_distribution<double> ua(-1.0, 1.0);
  for (int i = 0; i < 400000; i++) {
    const double b = std::floor(ua(g) * q);
    const double amax = std::min(std::floor(lim * q / std::max(1.0, std::fabs(b))), 3 * q);
    one(std::floor(ua(g) * amax), b);
  }
  std::printf("mulmod q=%.0f: %ld products exact in |a*b/q| < 2^51\n", q, n);
}

static void check_mulmod_c(double q, std::mt19937_64& g) {
  const double qi = 1.0 / q, lim = std::ldexp(1.0, 51);
  long n = 0, nbelow = 0, bad_below = 0;
  auto one = [&](double a, double w, bool twiddle_form) {
    const d2 t = twiddle_form ? fk::twiddle(w, qi) : d2{w, w / q};
    const double quo = a * w / q;
    if (!(std::fabs(a) < std::ldexp(1.0, 52))) return;
    const double r = fk::mulmod_c(a, t.x, t.y, q);
    if (quo <= -lim * (1 + 1e-12)) {   // outside the contract: count non-integer results
      nbelow++;
      if (!is_int(r) || !congruent_prod(r, a, w, q)) bad_below++;
      return;
    }
    if (!(quo > -lim * (1 - 1e-12))) return;
    n++;
    const double bound = (quo < lim * (1 - 1e-12) ? 0.5 : 1.0) * q + std::fabs(a) / 4.0;
    if (!is_int(r) || !congruent_prod(r, a, w, q) || !(std::fabs(r) <= bound)) fail("mulmod_c", a, w, q, r);
  };
  std::uniform_real_distribution<double> u01(0.0, 1.0), ua(-1.0, 1.0);
  std::vector<double> ws = {0, 1, 2, q - 1, q - 2, std::floor(q / 2), std::floor(q / 2) + 1};
  std::vector<double> as = {0, 1, -1, q - 1, -(q - 1), 2 * q - 1, -(2 * q - 1), 3 * q, -3 * q, 3.86 * q, 4.36 * q,
                            -1.9 * q, -2 * q + 1};
  for (int tf = 0; tf < 2; tf++) {
    for (double w : ws)
      for (double a : as) one(std::floor(a), w, tf);
    for (int i = 0; i < 300000; i++) {
      const double w = std::floor(u01(g) * q);
      one(std::floor(ua(g) * 4.4 * q), w, tf);
    }
  }
  std::printf("mulmod_c q=%.0f: %ld products exact for a*w/q > -2^51; %ld of %ld below -2^51 not exact\n", q, n,
              bad_below, nbelow);
  // the lower end of the band is where exactness ends: with a 50-bit q some
  // products below -2^51 must come out as non-integers
  if (q > std::ldexp(1.0, 49) && nbelow > 1000 && bad_below == 0) {
    std::printf("FAIL mulmod_c: no inexact product below -2^51 (precondition not tight?)\n");
    failures++;
  }
}

static void check_red_conv(double q, std::mt19937_64& g) {
  const double qi = 1.0 / q;
  std::uniform_real_distribution<double> ua(-1.0, 1.0);
  long n = 0;
  auto one = [&](double x) {
    const double r = fk::red(x, q, qi);
    n++;
    const i128 d = (i128)(int64_t)x - (i128)(int64_t)r;
    if (!is_int(r) || d % (i128)(int64_t)q != 0 || std::fabs(r) > q / 2 + 1) fail("red", x, 0, q, r);
    const double fn = fk::full_norm(x, q, qi);
    if (!is_int(fn) || fn < 0 || fn >= q || emod((i128)(int64_t)x, (i128)(int64_t)q) != (i128)(int64_t)fn)
      fail("full_norm", x, 0, q, fn);
  };
  const double big = std::ldexp(1.0, 52) - 1;
  for (double x : {0.0, 1.0, -1.0, q - 1, -(q - 1), q, -q, std::floor(q / 2), std::floor(q / 2) + 1, big, -big})
    one(x);
  for (int i = 0; i < 200000; i++) one(std::floor(ua(g) * big));
  for (int i = 0; i < 200000; i++) one(std::floor(ua(g) * 8 * q));
  // norm / centre on (-q, q)
  for (int i = 0; i < 100000; i++) {
    const double x = std::floor(ua(g) * (q - 1));
    const double nn = fk::norm(x, q), c = fk::centre(x, q);
    if (nn < 0 || nn >= q || emod((i128)(int64_t)(nn - x), (i128)(int64_t)q) != 0) fail("norm", x, 0, q, nn);
    if (std::fabs(c) > (q - 1) / 2 || emod((i128)(int64_t)(c - x), (i128)(int64_t)q) != 0) fail("centre", x, 0, q, c);
  }
  std::printf("red/full_norm q=%.0f: %ld values\n", q, n);
  std::uniform_int_distribution<uint64_t> uw(0, (1ull << 52) - 1);
  for (int i = 0; i < 200000; i++) {
    const uint64_t w = i < 4 ? (uint64_t[]){0, 1, (1ull << 52) - 1, 1ull << 51}[i] : uw(g);
    const double d = fk::u2d(w);
    if (d != (double)w || fk::d2u(d) != w) fail("u2d/d2u", (double)w, 0, 0, d);
  }
}

// Forward and inverse register rounds on a group of 2^K values with a
// caller-chosen twiddle per (stage, member), against exact integer butterflies.
template <int K>
static void check_rounds(double q, std::mt19937_64& g) {
  const int n = 1 << K;
  const double qi = 1.0 / q;
  const int64_t Q = (int64_t)q;
  std::uniform_int_distribution<int64_t> uq(0, Q - 1), uc(-(Q / 2), Q / 2);
  long cases = 0;
  auto run = [&](const std::vector<int64_t>& in, const std::vector<int64_t>& tw, bool fwd = true) {
    // tw[s * n + member] for stage s
    std::vector<double> v(n);
    for (int f = 0; f < n; f++) v[f] = (double)in[f];
    std::vector<double> out(n), outi(n);
    auto ld = [&](int i) { return v[i]; };
    auto st = [&](int i, double x) { out[i] = x; };
    auto twf = [&](int s, int idx) { return fk::twiddle((double)tw[s * n + idx], qi); };
    std::vector<i128> x(n);
    if (fwd) {
    fk::fwd_round<K>(0, 0, K, q, qi, ld, st, twf);
    // exact forward network: stage s pairs bit K-1-s; upper member a gets x_a + w x_b, lower x_a - w x_b
    for (int f = 0; f < n; f++) x[f] = in[f];
    for (int s = 0; s < K; s++) {
      const int half = 1 << (K - 1 - s);
      for (int f = 0; f < n; f++) {
        if (f & half) continue;
        const i128 t = emod(x[f | half] * (i128)tw[s * n + f], Q);
        const i128 u = x[f];
        x[f] = emod(u + t, Q);
        x[f | half] = emod(u - t, Q);
      }
    }
    for (int f = 0; f < n; f++)
      if (!is_int(out[f]) || emod((i128)(int64_t)out[f], Q) != x[f] || std::fabs(out[f]) > q / 2 + 1)
        fail(K == 3 ? "fwd_round<3>" : "fwd_round<4>", (double)in[f], (double)f, q, out[f]);
    }
    // inverse network: stage s pairs bit s; x_a + x_b, (x_a - x_b) w
    auto sti = [&](int i, double y) { outi[i] = y; };
    fk::inv_round<K>(0, 0, q, qi, ld, sti, twf);
    for (int f = 0; f < n; f++) x[f] = in[f];
    for (int s = 0; s < K; s++) {
      const int half = 1 << s;
      for (int f = 0; f < n; f++) {
        if (f & half) continue;
        const i128 a = x[f], b = x[f | half];
        x[f] = emod(a + b, Q);
        x[f | half] = emod((a - b) * (i128)tw[s * n + f], Q);
      }
    }
    for (int f = 0; f < n; f++)
      if (!is_int(outi[f]) || emod((i128)(int64_t)outi[f], Q) != x[f] || !(std::fabs(outi[f]) < q))
        fail(K == 3 ? "inv_round<3>" : "inv_round<4>", (double)in[f], (double)f, q, outi[f]);
    cases++;
  };
  auto run_inv = [&](const std::vector<int64_t>& in, const std::vector<int64_t>& tw) { run(in, tw, false); };
  std::vector<int64_t> in(n), tw(K * n);
  // adversarial: every input 0 or q-1 (HBM form) with every twiddle in {1, q-1, (q-1)/2}
  for (int64_t tv : {(int64_t)1, Q - 1, (Q - 1) / 2, (Q + 1) / 2})
    for (int pat = 0; pat < (1 << n) && pat < 65536; pat += (n == 16 ? 7 : 1)) {
      for (int f = 0; f < n; f++) in[f] = (pat >> f & 1) ? Q - 1 : 0;
      for (auto& t : tw) t = tv;
      run(in, tw);
    }
  // centred (LDS) inputs at +-q/2 with the same twiddles
  for (int64_t tv : {(int64_t)1, Q - 1, (Q - 1) / 2})
    for (int pat = 0; pat < (1 << n) && pat < 65536; pat += (n == 16 ? 7 : 1)) {
      for (int f = 0; f < n; f++) in[f] = (pat >> f & 1) ? Q / 2 + 1 : -(Q / 2 + 1);
      for (auto& t : tw) t = tv;
      run(in, tw);
    }
  // random inputs in both forms with random twiddles near the top of [0, q)
  std::uniform_int_distribution<int64_t> utop(Q - (Q >> 4), Q - 1);
  for (int i = 0; i < 60000; i++) {
    for (int f = 0; f < n; f++) in[f] = (i & 1) ? uq(g) : uc(g);
    for (auto& t : tw) t = (i & 2) ? utop(g) : uq(g);
    run(in, tw);
  }
  // the inverse rounds also take the previous round's outputs, anywhere in (-q, q)
  std::uniform_int_distribution<int64_t> uf(-(Q - 1), Q - 1);
  for (int i = 0; i < 20000; i++) {
    for (int f = 0; f < n; f++) in[f] = uf(g);
    for (auto& t : tw) t = (i & 2) ? utop(g) : uq(g);
    run_inv(in, tw);
  }
  std::printf("register rounds K=%d q=%.0f: %ld groups\n", K, q, cases);
}

int main() {
  std::mt19937_64 g(20261203);
  for (int bits : {30, 40, 50}) {
    const double q = (double)prime_below(bits, 17);
    check_mulmod(q, g);
    check_mulmod_c(q, g);
    check_red_conv(q, g);
    check_rounds<3>(q, g);
    check_rounds<4>(q, g);
  }
  std::printf("%s (%d failures)\n", failures ? "FAILED" : "ok", failures);
  return failures ? 1 : 0;
}
