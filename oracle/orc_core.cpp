// Oracle core: modular arithmetic, primes, negacyclic NTT, sampler, keys,
// encryption, hybrid key switching, rotations, rescale.  TEST INFRASTRUCTURE.
//
// Definitions followed (the paper builds on an existing CKKS library and only
// states the rotation formula; the substrate below is the standard full-RNS
// CKKS it relies on):
//   * Background section, CKKS primitives: Add, PMult, Rot, Rescale.
//   * Background section, eq. (rotation): Rot = automorphism + key switching
//     with the special modulus P and the scaling by P^{-1}.  Read as hybrid key
//     switching (Han-Ki, CT-RSA 2020) with dnum digits, ModUp/ModDown by the
//     fast base conversion of Bajard-Eynard-Hasan-Zucca (SAC 2016), and the
//     Galois element 5^r mod 2N for a left rotation by r slots.
//   * Rescale: division by the last prime with rounding to nearest
//     (Cheon-Han-Kim-Kim-Song, SAC 2018).
// Pins (tests/test_oracle_core.py): schoolbook negacyclic products, NTT
// round trip, Miller-Rabin against trial division, automorphism composition,
// ModUp/ModDown/rescale against big-integer CRT at toy sizes, decryption of
// rotated ciphertexts against numpy.roll.
#include "orc.h"
#include <quadmath.h>
#include <cassert>
#include <cmath>
#include <stdexcept>

namespace orc {

u64 powm(u64 a, u64 e, u64 q) {
  u64 r = 1 % q;
  a %= q;
  while (e) {
    if (e & 1) r = mulm(r, a, q);
    a = mulm(a, a, q);
    e >>= 1;
  }
  return r;
}

u64 invm(u64 a, u64 q) {
  a %= q;
  if (a == 0) throw std::runtime_error("invm: zero");
  return powm(a, q - 2, q);
}

bool is_prime(u64 n) {
  if (n < 2) return false;
  static const u64 small[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  for (u64 p : small) {
    if (n == p) return true;
    if (n % p == 0) return false;
  }
  u64 d = n - 1;
  int r = 0;
  while ((d & 1) == 0) { d >>= 1; r++; }
  for (u64 a : small) {
    u64 x = powm(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int i = 1; i < r; i++) {
      x = mulm(x, x, n);
      if (x == n - 1) { comp = false; break; }
    }
    if (comp) return false;
  }
  return true;
}

// ---------------------------------------------------------------- sampler
u64 mix64(u64 z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

u64 rng(u64 seed, u64 tag, u64 i) {
  u64 key = mix64(seed ^ (tag * 0xD1B54A32D192ED03ull));
  return mix64(key + (i + 1) * 0x9E3779B97F4A7C15ull);
}

int sample_ternary(u64 seed, u64 tag, u64 i) {
  u64 r = rng(seed, tag, i);
  return (int)(((u128)r * 3) >> 64) - 1;
}

u64 sample_uniform(u64 seed, u64 tag, u64 i, u64 q) {
  u64 hi = rng(seed, tag, 2 * i), lo = rng(seed, tag, 2 * i + 1);
  u128 v = ((u128)hi << 64) | lo;
  return (u64)(v % q);
}

// Cumulative table of the discrete Gaussian folded onto |e| (sigma = 3.2,
// support |e| <= 19): T[k-1] = floor(2^63 * P(|e| <= k-1)), k = 1..19.
const std::vector<u64>& gauss_cdt() {
  static const std::vector<u64> T = [] {   // built once (thread-safe static initialisation)
    std::vector<u64> t;
    const __float128 sigma = 3.2Q;
    __float128 rho[20];
    for (int k = 0; k < 20; k++) rho[k] = expq(-(__float128)(k * k) / (2 * sigma * sigma));
    __float128 Z = rho[0];
    for (int k = 1; k < 20; k++) Z += 2 * rho[k];
    __float128 cdf = rho[0] / Z;
    const __float128 two63 = ldexpq(1.0Q, 63);
    for (int k = 1; k < 20; k++) {
      t.push_back((u64)floorq(cdf * two63));
      cdf += 2 * rho[k] / Z;
    }
    return t;
  }();
  return T;
}

int sample_gauss(u64 seed, u64 tag, u64 i) {
  const std::vector<u64>& T = gauss_cdt();
  u64 r = rng(seed, tag, i);
  u64 sign = r >> 63, u = r & ((1ull << 63) - 1);
  int mag = 0;
  for (u64 t : T)
    if (u >= t) mag++;
  return sign ? -mag : mag;
}

// ---------------------------------------------------------------- ring
void cyclic_dft(Vec& a, const Vec& wpow, u64 q) {
  const size_t n = a.size();
  for (size_t i = 1, j = 0; i < n; i++) {
    size_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  for (size_t len = 2; len <= n; len <<= 1) {
    size_t step = n / len;
    for (size_t i = 0; i < n; i += len)
      for (size_t j = 0; j < len / 2; j++) {
        u64 u = a[i + j], v = mulm(a[i + j + len / 2], wpow[j * step], q);
        a[i + j] = addm(u, v, q);
        a[i + j + len / 2] = subm(u, v, q);
      }
  }
}

void Ring::init(int N_, u64 q_) {
  N = N_;
  q = q_;
  psi = find_psi(q, N);
  u64 psi_inv = invm(psi, q), om = mulm(psi, psi, q), om_inv = invm(om, q);
  psi_pow.resize(N);
  psi_inv_pow.resize(N);
  omega_pow.resize(N);
  omega_inv_pow.resize(N);
  u64 a = 1, b = 1, c = 1, d = 1;
  for (int i = 0; i < N; i++) {
    psi_pow[i] = a; psi_inv_pow[i] = b; omega_pow[i] = c; omega_inv_pow[i] = d;
    a = mulm(a, psi, q); b = mulm(b, psi_inv, q); c = mulm(c, om, q); d = mulm(d, om_inv, q);
  }
  n_inv = invm((u64)N, q);
}

void Ring::ntt(Vec& a) const {
  for (int i = 0; i < N; i++) a[i] = mulm(a[i], psi_pow[i], q);
  cyclic_dft(a, omega_pow, q);
}

void Ring::intt(Vec& a) const {
  cyclic_dft(a, omega_inv_pow, q);
  for (int i = 0; i < N; i++) a[i] = mulm(mulm(a[i], n_inv, q), psi_inv_pow[i], q);
}

Vec find_primes(int bits, int logN, int count, const Vec& taken) {
  Vec out;
  const u64 twoN = 2ull << logN;
  u64 k = ((1ull << bits) - 2) / twoN;
  while ((int)out.size() < count) {
    if (k == 0) throw std::runtime_error("find_primes: ran out of candidates");
    u64 p = k * twoN + 1;
    bool used = false;
    for (u64 t : taken) used |= (t == p);
    if (!used && is_prime(p)) out.push_back(p);
    k--;
  }
  return out;
}

u64 find_psi(u64 q, int N) {
  for (u64 x = 2;; x++) {
    u64 psi = powm(x, (q - 1) / (2 * (u64)N), q);
    if (powm(psi, (u64)N, q) == q - 1) return psi;
  }
}

Context::Context(const Params& p) : prm(p) {
  N = 1 << p.logN;
  ns = N / 2;
  L = p.nq - 1;
  K = p.np;
  alpha = (p.nq + p.dnum - 1) / p.dnum;
  Vec qs = find_primes(p.qbits, p.logN, p.nq, {});
  Vec ps = find_primes(p.pbits, p.logN, p.np, qs);
  primes = qs;
  primes.insert(primes.end(), ps.begin(), ps.end());
  ring.resize(primes.size());
  for (size_t i = 0; i < primes.size(); i++) ring[i].init(N, primes[i]);
  s.resize(N);
  for (int i = 0; i < N; i++) s[i] = sample_ternary(p.seed, TAG_SECRET, i);
}

u64 Context::galois(i64 shift) const {
  i64 r = shift % ns;
  if (r < 0) r += ns;
  return powm(5, (u64)r, 2 * (u64)N);
}

std::vector<int> q_basis(int level) {
  std::vector<int> v;
  for (int i = 0; i <= level; i++) v.push_back(i);
  return v;
}

std::vector<int> qp_basis(const Context& C, int level) {
  std::vector<int> v = q_basis(level);
  for (int k = 0; k < C.K; k++) v.push_back(C.L + 1 + k);
  return v;
}

// ---------------------------------------------------------------- polys
RPoly poly_zero(const Context& C, const std::vector<int>& pidx) {
  RPoly r;
  r.pidx = pidx;
  r.c.assign(pidx.size(), Vec(C.N, 0));
  return r;
}

RPoly poly_mul(const Context& C, const RPoly& a, const RPoly& b) {
  assert(a.pidx == b.pidx);
  RPoly r = poly_zero(C, a.pidx);
  for (size_t l = 0; l < a.pidx.size(); l++) {
    const Ring& R = C.ring[a.pidx[l]];
    Vec x = a.c[l], y = b.c[l];
    R.ntt(x);
    R.ntt(y);
    for (int i = 0; i < C.N; i++) x[i] = mulm(x[i], y[i], R.q);
    R.intt(x);
    r.c[l] = x;
  }
  return r;
}

RPoly poly_mul_schoolbook(const Context& C, const RPoly& a, const RPoly& b) {
  RPoly r = poly_zero(C, a.pidx);
  const int N = C.N;
  for (size_t l = 0; l < a.pidx.size(); l++) {
    u64 q = C.primes[a.pidx[l]];
    for (int i = 0; i < N; i++)
      for (int j = 0; j < N; j++) {
        u64 t = mulm(a.c[l][i], b.c[l][j], q);
        int k = i + j;
        if (k < N) r.c[l][k] = addm(r.c[l][k], t, q);
        else r.c[l][k - N] = subm(r.c[l][k - N], t, q);   // X^N = -1
      }
  }
  return r;
}

void poly_add_inplace(const Context& C, RPoly& a, const RPoly& b) {
  assert(a.pidx == b.pidx);
  for (size_t l = 0; l < a.pidx.size(); l++) {
    u64 q = C.primes[a.pidx[l]];
    for (int i = 0; i < C.N; i++) a.c[l][i] = addm(a.c[l][i], b.c[l][i], q);
  }
}

void poly_sub_inplace(const Context& C, RPoly& a, const RPoly& b) {
  assert(a.pidx == b.pidx);
  for (size_t l = 0; l < a.pidx.size(); l++) {
    u64 q = C.primes[a.pidx[l]];
    for (int i = 0; i < C.N; i++) a.c[l][i] = subm(a.c[l][i], b.c[l][i], q);
  }
}

RPoly poly_scalar(const Context& C, const RPoly& a, i64 s) {
  RPoly r = a;
  for (size_t l = 0; l < a.pidx.size(); l++) {
    u64 q = C.primes[a.pidx[l]], sm = from_i64(s, q);
    for (int i = 0; i < C.N; i++) r.c[l][i] = mulm(a.c[l][i], sm, q);
  }
  return r;
}

// sigma_g: coefficient i moves to index i*g mod 2N, negated when that index is >= N
RPoly automorph(const Context& C, const RPoly& a, u64 g) {
  RPoly r = poly_zero(C, a.pidx);
  const u64 N = C.N, twoN = 2 * N;
  for (size_t l = 0; l < a.pidx.size(); l++) {
    u64 q = C.primes[a.pidx[l]];
    for (u64 i = 0; i < N; i++) {
      u64 k = (i * g) % twoN;
      if (k < N) r.c[l][k] = a.c[l][i];
      else r.c[l][k - N] = negm(a.c[l][i], q);
    }
  }
  return r;
}

// ---------------------------------------------------------------- secret
RPoly secret_poly(const Context& C, const std::vector<int>& pidx) {
  RPoly r = poly_zero(C, pidx);
  for (size_t l = 0; l < pidx.size(); l++) {
    u64 q = C.primes[pidx[l]];
    for (int i = 0; i < C.N; i++) r.c[l][i] = from_i64(C.s[i], q);
  }
  return r;
}

RPoly secret_square_poly(const Context& C, const std::vector<int>& pidx) {
  RPoly s = secret_poly(C, pidx);
  return poly_mul(C, s, s);
}

static u64 prod_p_mod(const Context& C, u64 q) {
  u64 r = 1 % q;
  for (int k = 0; k < C.K; k++) r = mulm(r, C.primes[C.L + 1 + k] % q, q);
  return r;
}

std::vector<std::vector<RPoly>> gen_switch_key(Context& C, u64 keyid) {
  const std::vector<int> basis = qp_basis(C, C.L);
  RPoly s = secret_poly(C, basis);
  RPoly target = (keyid == 0) ? secret_square_poly(C, basis) : automorph(C, s, keyid);
  const int ndig = (C.L + 1 + C.alpha - 1) / C.alpha;
  std::vector<std::vector<RPoly>> key(ndig);
  for (int j = 0; j < ndig; j++) {
    const int lo = j * C.alpha, hi = std::min((j + 1) * C.alpha, C.L + 1);
    RPoly a = poly_zero(C, basis), e = poly_zero(C, basis);
    for (size_t l = 0; l < basis.size(); l++) {
      int pi = basis[l];
      u64 q = C.primes[pi];
      for (int i = 0; i < C.N; i++) {
        a.c[l][i] = sample_uniform(C.prm.seed, tag_key_a(keyid, j, pi), i, q);
        e.c[l][i] = from_i64(sample_gauss(C.prm.seed, tag_key_e(keyid, j), i), q);
      }
    }
    RPoly b = poly_mul(C, a, s);
    RPoly nb = poly_zero(C, basis);
    poly_sub_inplace(C, nb, b);          // -a*s
    poly_add_inplace(C, nb, e);          // -a*s + e
    for (size_t l = 0; l < basis.size(); l++) {
      int pi = basis[l];
      if (pi < lo || pi >= hi) continue;   // gadget only on the digit's own primes
      u64 q = C.primes[pi], Pq = prod_p_mod(C, q);
      for (int i = 0; i < C.N; i++) nb.c[l][i] = addm(nb.c[l][i], mulm(Pq, target.c[l][i], q), q);
    }
    key[j] = {nb, a};
  }
  return key;
}

const std::vector<std::vector<std::vector<Vec>>>& Context::key(u64 keyid) {
  // The map lock covers only finding or adding the key's slot; each key is
  // generated once (its own once-flag), distinct keys concurrently.  Slots
  // are never removed, so the reference stays valid.
  KeySlot* slot;
  {
    std::lock_guard<std::mutex> lock(*key_mu);
    auto& p = keys[keyid];
    if (!p) p = std::make_shared<KeySlot>();
    slot = p.get();
  }
  std::call_once(slot->once, [&] {
    std::vector<std::vector<RPoly>> k = gen_switch_key(*this, keyid);
    std::vector<std::vector<std::vector<Vec>>> kn(k.size());
    for (size_t j = 0; j < k.size(); j++) {
      kn[j].resize(2);
      for (int t = 0; t < 2; t++) {
        kn[j][t].resize(primes.size());
        const RPoly& P = k[j][t];
        for (size_t l = 0; l < P.pidx.size(); l++) {
          Vec v = P.c[l];
          ring[P.pidx[l]].ntt(v);
          kn[j][t][P.pidx[l]] = v;
        }
      }
    }
    slot->key = std::move(kn);
  });
  return slot->key;
}

// ---------------------------------------------------------------- encryption
Ct encrypt(const Context& C, const RPoly& pt, int level, double scale, u64 enc_seed, u64 ct_index) {
  std::vector<int> basis = q_basis(level);
  RPoly a = poly_zero(C, basis), e = poly_zero(C, basis);
  for (int l = 0; l <= level; l++) {
    u64 q = C.primes[l];
    for (int i = 0; i < C.N; i++) {
      a.c[l][i] = sample_uniform(enc_seed, tag_enc_a(ct_index, l), i, q);
      e.c[l][i] = from_i64(sample_gauss(enc_seed, tag_enc_e(ct_index), i), q);
    }
  }
  RPoly s = secret_poly(C, basis);
  Ct ct;
  ct.c0 = poly_zero(C, basis);
  poly_sub_inplace(C, ct.c0, poly_mul(C, a, s));
  poly_add_inplace(C, ct.c0, e);
  poly_add_inplace(C, ct.c0, pt);
  ct.c1 = a;
  ct.level = level;
  ct.scale = scale;
  return ct;
}

RPoly decrypt(const Context& C, const Ct& ct) {
  RPoly s = secret_poly(C, ct.c0.pidx);
  RPoly m = poly_mul(C, ct.c1, s);
  poly_add_inplace(C, m, ct.c0);
  return m;
}

// ---------------------------------------------------------------- key switching
std::vector<RPoly> mod_up(const Context& C, const RPoly& d, int level) {
  const std::vector<int> ext = qp_basis(C, level);
  const int beta = (level + 1 + C.alpha - 1) / C.alpha;
  std::vector<RPoly> out;
  for (int j = 0; j < beta; j++) {
    const int lo = j * C.alpha, hi = std::min((j + 1) * C.alpha, level + 1);
    // y_i = [d_i * (Qj/q_i)^{-1}]_{q_i}, centred in (-q_i/2, q_i/2]
    std::vector<std::vector<i64>> y(hi - lo, std::vector<i64>(C.N));
    for (int i = lo; i < hi; i++) {
      u64 qi = C.primes[i], hat = 1;
      for (int i2 = lo; i2 < hi; i2++)
        if (i2 != i) hat = mulm(hat, C.primes[i2] % qi, qi);
      u64 hinv = invm(hat, qi);
      for (int c = 0; c < C.N; c++) {
        u64 v = mulm(d.c[i][c], hinv, qi);
        y[i - lo][c] = v <= (qi - 1) / 2 ? (i64)v : (i64)v - (i64)qi;
      }
    }
    RPoly r = poly_zero(C, ext);
    for (size_t l = 0; l < ext.size(); l++) {
      int t = ext[l];
      if (t >= lo && t < hi) {   // the digit's own limbs are copied
        r.c[l] = d.c[t];
        continue;
      }
      u64 qt = C.primes[t];
      for (int i = lo; i < hi; i++) {
        u64 hat = 1;   // [Qj / q_i]_t
        for (int i2 = lo; i2 < hi; i2++)
          if (i2 != i) hat = mulm(hat, C.primes[i2] % qt, qt);
        for (int c = 0; c < C.N; c++) r.c[l][c] = addm(r.c[l][c], mulm(from_i64(y[i - lo][c], qt), hat, qt), qt);
      }
    }
    out.push_back(r);
  }
  return out;
}

RPoly mod_down(const Context& C, const RPoly& a, int level) {
  RPoly r = poly_zero(C, q_basis(level));
  const int off = level + 1;   // P limbs follow the level+1 Q limbs in qp_basis
  // y_k = [a_{p_k} (P/p_k)^{-1}]_{p_k}, centred in (-p_k/2, p_k/2]
  std::vector<std::vector<i64>> y(C.K, std::vector<i64>(C.N));
  for (int k = 0; k < C.K; k++) {
    u64 pk = C.primes[C.L + 1 + k], hat = 1;
    for (int k2 = 0; k2 < C.K; k2++)
      if (k2 != k) hat = mulm(hat, C.primes[C.L + 1 + k2] % pk, pk);
    u64 hinv = invm(hat, pk);
    for (int c = 0; c < C.N; c++) {
      u64 v = mulm(a.c[off + k][c], hinv, pk);
      y[k][c] = v <= (pk - 1) / 2 ? (i64)v : (i64)v - (i64)pk;
    }
  }
  for (int i = 0; i <= level; i++) {
    u64 qi = C.primes[i];
    u64 Pinv = invm(prod_p_mod(C, qi), qi);
    std::vector<u64> hat(C.K);
    for (int k = 0; k < C.K; k++) {
      hat[k] = 1;
      for (int k2 = 0; k2 < C.K; k2++)
        if (k2 != k) hat[k] = mulm(hat[k], C.primes[C.L + 1 + k2] % qi, qi);
    }
    for (int c = 0; c < C.N; c++) {
      u64 conv = 0;
      for (int k = 0; k < C.K; k++) conv = addm(conv, mulm(from_i64(y[k][c], qi), hat[k], qi), qi);
      r.c[i][c] = mulm(subm(a.c[i][c], conv, qi), Pinv, qi);
    }
  }
  return r;
}

void key_inner_product(Context& C, const std::vector<RPoly>& ext, u64 keyid, int level,
                       RPoly& acc0, RPoly& acc1) {
  const auto& key = C.key(keyid);
  const std::vector<int> basis = qp_basis(C, level);
  acc0 = poly_zero(C, basis);
  acc1 = poly_zero(C, basis);
  for (size_t l = 0; l < basis.size(); l++) {
    const int pi = basis[l];
    const Ring& R = C.ring[pi];
    Vec s0(C.N, 0), s1(C.N, 0);
    for (size_t j = 0; j < ext.size(); j++) {
      Vec x = ext[j].c[l];
      R.ntt(x);
      for (int i = 0; i < C.N; i++) {
        s0[i] = addm(s0[i], mulm(x[i], key[j][0][pi][i], R.q), R.q);
        s1[i] = addm(s1[i], mulm(x[i], key[j][1][pi][i], R.q), R.q);
      }
    }
    R.intt(s0);
    R.intt(s1);
    acc0.c[l] = s0;
    acc1.c[l] = s1;
  }
}

std::vector<Ct> rotate_hoisted(Context& C, const Ct& x, const std::vector<i64>& shifts) {
  std::vector<RPoly> ext = mod_up(C, x.c1, x.level);
  std::vector<Ct> out(shifts.size());
  par_for((int)shifts.size(), [&](int k) {   // the shifts share the ModUp and nothing else
    u64 g = C.galois(shifts[k]);
    if (g == 1) throw std::runtime_error("rotate_hoisted: zero shift");
    std::vector<RPoly> eg;
    for (const RPoly& e : ext) eg.push_back(automorph(C, e, g));
    RPoly a0, a1;
    key_inner_product(C, eg, g, x.level, a0, a1);
    Ct y;
    y.c0 = automorph(C, x.c0, g);
    poly_add_inplace(C, y.c0, mod_down(C, a0, x.level));
    y.c1 = mod_down(C, a1, x.level);
    y.level = x.level;
    y.scale = x.scale;
    out[k] = y;
  });
  return out;
}

// P mod q for every prime index of pidx (zero on the special primes)
static std::vector<u64> p_mod(const Context& C, const std::vector<int>& pidx) {
  std::vector<u64> r;
  for (int i : pidx) {
    const u64 q = C.primes[i];
    u64 v = 1;
    for (int k = 0; k < C.K; k++) v = mulm(v, C.primes[C.L + 1 + k] % q, q);
    r.push_back(v);
  }
  return r;
}

std::vector<Ct> rotate_hoisted_pq(Context& C, const Ct& x, const std::vector<i64>& shifts) {
  std::vector<RPoly> ext = mod_up(C, x.c1, x.level);
  const std::vector<int> qp = qp_basis(C, x.level);
  const std::vector<u64> pm = p_mod(C, qp);
  std::vector<Ct> out(shifts.size());
  par_for((int)shifts.size(), [&](int k) {   // the shifts share the ModUp and nothing else
    u64 g = C.galois(shifts[k]);
    if (g == 1) throw std::runtime_error("rotate_hoisted_pq: zero shift");
    std::vector<RPoly> eg;
    for (const RPoly& e : ext) eg.push_back(automorph(C, e, g));
    RPoly a0, a1;
    key_inner_product(C, eg, g, x.level, a0, a1);
    const RPoly c0g = automorph(C, x.c0, g);
    for (int l = 0; l <= x.level; l++) {   // + P sigma_g(c0) on the Q limbs (P = 0 mod p_k)
      const u64 q = C.primes[qp[l]];
      for (int i = 0; i < C.N; i++) a0.c[l][i] = addm(a0.c[l][i], mulm(c0g.c[l][i], pm[l], q), q);
    }
    Ct y;
    y.c0 = a0;
    y.c1 = a1;
    y.level = x.level;
    y.scale = x.scale;
    out[k] = y;
  });
  return out;
}

Ct lift_pq(const Context& C, const Ct& x) {
  const std::vector<int> qp = qp_basis(C, x.level);
  const std::vector<u64> pm = p_mod(C, qp);
  Ct y;
  y.c0 = poly_zero(C, qp);
  y.c1 = poly_zero(C, qp);
  for (int l = 0; l <= x.level; l++) {
    const u64 q = C.primes[qp[l]];
    for (int i = 0; i < C.N; i++) {
      y.c0.c[l][i] = mulm(x.c0.c[l][i], pm[l], q);
      y.c1.c[l][i] = mulm(x.c1.c[l][i], pm[l], q);
    }
  }
  y.level = x.level;
  y.scale = x.scale;
  return y;
}

Ct mod_down_ct(const Context& C, const Ct& y) {
  Ct r;
  r.c0 = mod_down(C, y.c0, y.level);
  r.c1 = mod_down(C, y.c1, y.level);
  r.level = y.level;
  r.scale = y.scale;
  return r;
}

Ct rotate_sum_lazy(Context& C, const Ct* z0, const std::vector<const Ct*>& zs,
                   const std::vector<i64>& shifts) {
  assert(!zs.empty() && zs.size() == shifts.size());
  const int level = zs[0]->level;
  const std::vector<int> qb = q_basis(level), ext = qp_basis(C, level);
  RPoly acc0 = poly_zero(C, ext), acc1 = poly_zero(C, ext);
  Ct y;
  y.c0 = z0 ? z0->c0 : poly_zero(C, qb);
  y.c1 = z0 ? z0->c1 : poly_zero(C, qb);
  // every term's ModUp and inner product are independent; the sums follow in term order
  std::vector<RPoly> k0(zs.size()), k1(zs.size());
  par_for((int)zs.size(), [&](int r) {
    u64 g = C.galois(shifts[r]);
    if (g == 1) throw std::runtime_error("rotate_sum_lazy: zero shift");
    std::vector<RPoly> up = mod_up(C, zs[r]->c1, level);
    for (RPoly& e : up) e = automorph(C, e, g);
    key_inner_product(C, up, g, level, k0[r], k1[r]);
  });
  for (size_t r = 0; r < zs.size(); r++) {
    poly_add_inplace(C, acc0, k0[r]);
    poly_add_inplace(C, acc1, k1[r]);
    poly_add_inplace(C, y.c0, automorph(C, zs[r]->c0, C.galois(shifts[r])));
  }
  poly_add_inplace(C, y.c0, mod_down(C, acc0, level));
  poly_add_inplace(C, y.c1, mod_down(C, acc1, level));
  y.level = level;
  y.scale = z0 ? z0->scale : zs[0]->scale;
  return y;
}

static RPoly rescale_poly(const Context& C, const RPoly& a, int level) {
  RPoly r = poly_zero(C, q_basis(level - 1));
  const u64 ql = C.primes[level];
  for (int i = 0; i < level; i++) {
    u64 qi = C.primes[i], inv = invm(ql % qi, qi);
    for (int c = 0; c < C.N; c++) {
      u64 last = a.c[level][c];
      i64 v = (last <= (ql - 1) / 2) ? (i64)last : (i64)last - (i64)ql;   // centred
      r.c[i][c] = mulm(subm(a.c[i][c], from_i64(v, qi), qi), inv, qi);
    }
  }
  return r;
}

Ct rescale(const Context& C, const Ct& x) {
  if (x.level == 0) throw std::runtime_error("rescale: level 0");
  Ct y;
  y.c0 = rescale_poly(C, x.c0, x.level);
  y.c1 = rescale_poly(C, x.c1, x.level);
  y.level = x.level - 1;
  y.scale = x.scale / (double)C.primes[x.level];
  return y;
}

Ct add(const Context& C, const Ct& a, const Ct& b) {
  if (a.level != b.level) throw std::runtime_error("add: level mismatch");
  Ct y = a;
  poly_add_inplace(C, y.c0, b.c0);
  poly_add_inplace(C, y.c1, b.c1);
  return y;
}

Ct mul_plain(const Context& C, const Ct& a, const RPoly& pt, double pt_scale) {
  Ct y;
  y.c0 = poly_mul(C, a.c0, pt);
  y.c1 = poly_mul(C, a.c1, pt);
  y.level = a.level;
  y.scale = a.scale * pt_scale;
  return y;
}

Ct mul_scalar(const Context& C, const Ct& a, i64 s, double s_scale) {
  Ct y;
  y.c0 = poly_scalar(C, a.c0, s);
  y.c1 = poly_scalar(C, a.c1, s);
  y.level = a.level;
  y.scale = a.scale * s_scale;
  return y;
}

Ct square_relin(Context& C, const Ct& a, i64 k) {
  RPoly d0 = poly_scalar(C, poly_mul(C, a.c0, a.c0), k);
  RPoly d1 = poly_scalar(C, poly_mul(C, a.c0, a.c1), 2 * k);
  RPoly d2 = poly_scalar(C, poly_mul(C, a.c1, a.c1), k);
  std::vector<RPoly> up = mod_up(C, d2, a.level);
  RPoly a0, a1;
  key_inner_product(C, up, 0, a.level, a0, a1);
  Ct y;
  y.c0 = d0;
  poly_add_inplace(C, y.c0, mod_down(C, a0, a.level));
  y.c1 = d1;
  poly_add_inplace(C, y.c1, mod_down(C, a1, a.level));
  y.level = a.level;
  y.scale = ((double)k * a.scale) * a.scale;
  return y;
}

Ct mul_relin(Context& C, const Ct& a, const Ct& b) {
  if (a.level != b.level) throw std::runtime_error("mul_relin: level mismatch");
  RPoly d0 = poly_mul(C, a.c0, b.c0);
  RPoly d1 = poly_mul(C, a.c0, b.c1);
  poly_add_inplace(C, d1, poly_mul(C, a.c1, b.c0));
  RPoly d2 = poly_mul(C, a.c1, b.c1);
  std::vector<RPoly> up = mod_up(C, d2, a.level);
  RPoly a0, a1;
  key_inner_product(C, up, 0, a.level, a0, a1);
  Ct y;
  y.c0 = d0;
  poly_add_inplace(C, y.c0, mod_down(C, a0, a.level));
  y.c1 = d1;
  poly_add_inplace(C, y.c1, mod_down(C, a1, a.level));
  y.level = a.level;
  y.scale = a.scale * b.scale;
  return y;
}

// ModDown by P q_l (Q_l U P -> Q_{l-1}): the special primes and q_l dropped
// by one fast base conversion, i.e. the ModDown of a relinearisation and the
// rescale after it taken together.  With D = P q_l and d_k its primes,
// y_k = [a_{d_k} (D/d_k)^-1]_{d_k} centred and
// out_i = (a_i - sum_k y_k [D/d_k]_{q_i}) D^-1 mod q_i, i < l.
RPoly mod_down_rescale(const Context& C, const RPoly& a, int level) {
  if (level < 1) throw std::runtime_error("mod_down_rescale: level 0");
  const int K = C.K;
  std::vector<u64> dp(K + 1);
  std::vector<int> row(K + 1);   // rows of the dropped primes in the qp basis of `level`
  dp[0] = C.primes[level];
  row[0] = level;
  for (int k = 0; k < K; k++) {
    dp[k + 1] = C.primes[C.L + 1 + k];
    row[k + 1] = level + 1 + k;
  }
  std::vector<std::vector<i64>> y(K + 1, std::vector<i64>(C.N));
  for (int k = 0; k <= K; k++) {
    const u64 d = dp[k];
    u64 hat = 1;
    for (int k2 = 0; k2 <= K; k2++)
      if (k2 != k) hat = mulm(hat, dp[k2] % d, d);
    const u64 hinv = invm(hat, d);
    for (int c = 0; c < C.N; c++) {
      const u64 v = mulm(a.c[row[k]][c], hinv, d);
      y[k][c] = v <= (d - 1) / 2 ? (i64)v : (i64)v - (i64)d;
    }
  }
  RPoly r = poly_zero(C, q_basis(level - 1));
  for (int i = 0; i < level; i++) {
    const u64 qi = C.primes[i];
    u64 D = 1;
    std::vector<u64> hat(K + 1, 1);
    for (int k = 0; k <= K; k++) {
      D = mulm(D, dp[k] % qi, qi);
      for (int k2 = 0; k2 <= K; k2++)
        if (k2 != k) hat[k] = mulm(hat[k], dp[k2] % qi, qi);
    }
    const u64 Dinv = invm(D, qi);
    for (int c = 0; c < C.N; c++) {
      u64 conv = 0;
      for (int k = 0; k <= K; k++) conv = addm(conv, mulm(from_i64(y[k][c], qi), hat[k], qi), qi);
      r.c[i][c] = mulm(subm(a.c[i][c], conv, qi), Dinv, qi);
    }
  }
  return r;
}

void tensor(const Context& C, const Ct& a, const Ct& b, i64 k, RPoly& d0, RPoly& d1, RPoly& d2) {
  if (a.level != b.level) throw std::runtime_error("tensor: level mismatch");
  d0 = poly_scalar(C, poly_mul(C, a.c0, b.c0), k);
  d1 = poly_mul(C, a.c0, b.c1);
  poly_add_inplace(C, d1, poly_mul(C, a.c1, b.c0));
  d1 = poly_scalar(C, d1, k);
  d2 = poly_scalar(C, poly_mul(C, a.c1, b.c1), k);
}

Ct relin_rescale(Context& C, const Ct& d, const RPoly& d2) {
  const int level = d.level;
  if (level < 1) throw std::runtime_error("relin_rescale: level 0");
  std::vector<RPoly> up = mod_up(C, d2, level);
  RPoly a0, a1;
  key_inner_product(C, up, 0, level, a0, a1);
  for (int l = 0; l <= level; l++) {   // + P (d0, d1) on the Q limbs; P is zero on the special primes
    const u64 q = C.primes[l], Pq = prod_p_mod(C, q);
    for (int c = 0; c < C.N; c++) {
      a0.c[l][c] = addm(a0.c[l][c], mulm(d.c0.c[l][c], Pq, q), q);
      a1.c[l][c] = addm(a1.c[l][c], mulm(d.c1.c[l][c], Pq, q), q);
    }
  }
  Ct y;
  y.c0 = mod_down_rescale(C, a0, level);
  y.c1 = mod_down_rescale(C, a1, level);
  y.level = level - 1;
  y.scale = d.scale / (double)C.primes[level];
  return y;
}

Ct drop_last_limb(const Ct& a) {
  if (a.level < 1) throw std::runtime_error("drop_last_limb: level 0");
  Ct y = a;
  y.c0.pidx.pop_back();
  y.c0.c.pop_back();
  y.c1.pidx.pop_back();
  y.c1.c.pop_back();
  y.level = a.level - 1;
  return y;
}

Ct lin_comb(const Context& C, const Ct* base, const Ct& x, i128 k1, i128 k0) {
  Ct y;
  y.level = x.level;
  y.scale = x.scale;
  y.c0 = poly_zero(C, x.c0.pidx);
  y.c1 = poly_zero(C, x.c1.pidx);
  for (size_t l = 0; l < x.c0.pidx.size(); l++) {
    const u64 q = C.primes[x.c0.pidx[l]], m = from_i128(k1, q);
    for (int i = 0; i < C.N; i++) {
      y.c0.c[l][i] = mulm(x.c0.c[l][i], m, q);
      y.c1.c[l][i] = mulm(x.c1.c[l][i], m, q);
    }
    y.c0.c[l][0] = addm(y.c0.c[l][0], from_i128(k0, q), q);
  }
  if (base) {
    poly_add_inplace(C, y.c0, base->c0);
    poly_add_inplace(C, y.c1, base->c1);
  }
  return y;
}

}  // namespace orc
