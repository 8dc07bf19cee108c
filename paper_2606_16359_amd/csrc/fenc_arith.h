// Exact 50-bit modular arithmetic on binary64 FMA, shared by every kernel.
//
// CDNA4 issues binary64 FMA at full rate but 32-bit integer multiplies at a
// quarter rate, so residues modulo primes q < 2^50 are handled as exact
// integers held in doubles:
//   * the product a*b is split exactly into h + l with h = fl(a*b),
//     l = fma(a, b, -h)  (Dekker's two-product via FMA);
//   * the quotient estimate e is formed in one FMA against the constant
//     1.5*2^52: fl(h*(1/q) + 1.5*2^52) - 1.5*2^52;
//   * r = fma(-e, q, h) + l = a*b - e*q, exact whenever e is an integer.
//
// Contract (checked against 128-bit integers by tests/test_arith.py):
//   The estimate is an integer exactly when the quotient a*b/q lies above
//   -2^51: on [-2^51, 2^51) the FMA result lies in [2^52, 2^53), where
//   doubles are the integers, and e is the nearest integer to fl(h/q) (off
//   by at most 1/2 + |a*b/q| 2^-52 from a*b/q); on [2^51, 2^52) it lies in
//   [2^53, 2^54) and e is the nearest even integer (off by at most 1 +
//   |a*b/q| 2^-52).  Below -2^51 the FMA result falls under 2^52, e can be a
//   half-integer and r is then not a residue at all.  So:
//     mulmod(a, b):      exact and |r| < q for |a*b/q| < 2^51;
//     mulmod_c(a, w):    w in [0, q), wq = fl(w/q) or fl(w * fl(1/q)); exact
//                        for a*w/q > -2^51 and |a| < 2^52, with
//                        |r| <= (1/2 + |a|/(4q)) q for a*w/q < 2^51 and
//                        |r| <= (1 + |a|/(4q)) q above;
//     red(x):            exact, |r| <= q/2 + 1, for |x| < 2^52.
//   With |b| < q, |a| < 2^51 is enough for mulmod (for q near 2^50 that is
//   |a| < 2q, not 3q).  Every call site states the operand range it relies on.
// Residues are stored in HBM as uint64 in [0, q) and converted with the
// 2^52 exponent trick (exact for values below 2^52).
#pragma once
#include <cstdint>
#include <cmath>

#ifndef FENC_HD
#define FENC_HD
#endif

namespace fk {

typedef uint64_t u64;

constexpr double kRound = 6755399441055744.0;   // 1.5 * 2^52
constexpr double kTwo52 = 4503599627370496.0;   // 2^52
constexpr u64 kExp52 = 0x4330000000000000ull;   // bit pattern of 2^52

FENC_HD inline double u2d(u64 x) { return __builtin_bit_cast(double, x | kExp52) - kTwo52; }
FENC_HD inline u64 d2u(double d) { return __builtin_bit_cast(u64, d + kTwo52) & 0x000FFFFFFFFFFFFFull; }

// integer nearest to x (|x| < 2^51)
FENC_HD inline double rint52(double x) { return (x + kRound) - kRound; }

// a*b mod q in (-q, q) for |a*b/q| < 2^51 (|a| < 2^51 with |b| < q)
FENC_HD inline double mulmod(double a, double b, double q, double qinv) {
  double h = a * b;
  double l = fma(a, b, -h);
  double e = fma(h, qinv, kRound) - kRound;
  return fma(-e, q, h) + l;
}

// a*w - e*q for a constant w in [0, q) with wq = fl(w/q); exact for
// a*w/q > -2^51, |a| < 2^52; magnitude bounds in the header comment
FENC_HD inline double mulmod_c(double a, double w, double wq, double q) {
  double h = a * w;
  double l = fma(a, w, -h);
  double e = fma(a, wq, kRound) - kRound;
  return fma(-e, q, h) + l;
}

// x mod q in [-q/2, q/2] (up to one unit); exact for |x| < 2^52
FENC_HD inline double red(double x, double q, double qinv) {
  double e = fma(x, qinv, kRound) - kRound;
  return fma(-e, q, x);
}

// representative in [0, q) of x in (-q, q)
FENC_HD inline double norm(double x, double q) { return x < 0 ? x + q : x; }
// centred representative in [-(q-1)/2, (q-1)/2] of x in (-q, q)
FENC_HD inline double centre(double x, double q) {
  const double t = x < 0 ? x + q : x;
  return t > (q - 1) * 0.5 ? t - q : t;
}
// representative in [0, q) of any |x| < 2^52
FENC_HD inline double full_norm(double x, double q, double qinv) {
  double r = red(x, q, qinv);
  r = r < 0 ? r + q : r;
  return r >= q ? r - q : r;
}

FENC_HD inline unsigned brev(unsigned x, int bits) {
  x = ((x >> 1) & 0x55555555u) | ((x & 0x55555555u) << 1);
  x = ((x >> 2) & 0x33333333u) | ((x & 0x33333333u) << 2);
  x = ((x >> 4) & 0x0F0F0F0Fu) | ((x & 0x0F0F0F0Fu) << 4);
  x = ((x >> 8) & 0x00FF00FFu) | ((x & 0x00FF00FFu) << 8);
  x = (x >> 16) | (x << 16);
  return bits ? x >> (32 - bits) : 0;
}

// Index permutation of the automorphism X -> X^g on an NTT vector stored in
// bit-reversed order (slot k holds the evaluation at psi^(2 brev(k) + 1)):
// out[k] = in[auto_src(k)].
FENC_HD inline unsigned auto_src(unsigned k, unsigned g, int logn) {
  const unsigned mask2n = (2u << logn) - 1;
  unsigned e = 2 * brev(k, logn) + 1;
  unsigned f = (unsigned)(((unsigned long long)e * g) & mask2n);
  return brev((f - 1) >> 1, logn);
}

}  // namespace fk
