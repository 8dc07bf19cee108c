// Oracle: CKKS canonical-embedding encoder/decoder in __float128.
// TEST INFRASTRUCTURE.
//
// Definition (Cheon-Kim-Kim-Song 2017, the encoding the paper's CKKS
// background section relies on): slot j holds m(zeta^{5^j}) / Delta with
// zeta = exp(i*pi/N); a plaintext is round(Delta * tau^{-1}(z)), rounding
// half away from zero.  tau^{-1} is evaluated as an inverse twisted DFT of
// size N over all primitive 2N-th roots (slot values on the 5^j roots, their
// conjugates on the -5^j roots).  Quad precision makes the computed value
// accurate to far below 1e-10 at the magnitudes used (< 2^53), so the rounding
// decision is the exact one except on a vanishing set of inputs.
// Pins: direct O(N^2) evaluation of the definition at N <= 64, decode(encode)
// round trip, a constant slot vector encodes to a constant polynomial.
#include "orc.h"
#include <quadmath.h>
#include <stdexcept>

namespace orc {

typedef __complex128 cq;

static cq expi(__float128 ang) {
  cq z;
  __real__ z = cosq(ang);
  __imag__ z = sinq(ang);
  return z;
}

// in-place radix-2 DFT of size n, sign -1 or +1 in the exponent, no scaling
static void fft_q(std::vector<cq>& a, int sign) {
  const size_t n = a.size();
  for (size_t i = 1, j = 0; i < n; i++) {
    size_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  for (size_t len = 2; len <= n; len <<= 1) {
    std::vector<cq> w(len / 2);
    for (size_t k = 0; k < len / 2; k++) w[k] = expi(sign * 2 * M_PIq * (__float128)k / (__float128)len);
    for (size_t i = 0; i < n; i += len)
      for (size_t k = 0; k < len / 2; k++) {
        cq u = a[i + k], v = a[i + k + len / 2] * w[k];
        a[i + k] = u + v;
        a[i + k + len / 2] = u - v;
      }
  }
}

static i64 round_half_away(__float128 v) {
  __float128 r = floorq(fabsq(v) + 0.5Q);
  if (r > ldexpq(1.0Q, 62)) throw std::runtime_error("encode: coefficient too large");
  i64 m = (i64)r;
  return v < 0 ? -m : m;
}

// E[t] for t in [0, N): evaluation of m at zeta^{2t+1}
static std::vector<cq> slots_to_evals(const Context& C, const std::vector<double>& re,
                                      const std::vector<double>& im) {
  const u64 twoN = 2 * (u64)C.N;
  std::vector<cq> E(C.N);
  for (int t = 0; t < C.N; t++) E[t] = 0;
  u64 e = 1;
  for (int j = 0; j < C.ns; j++) {
    cq z;
    __real__ z = (__float128)re[j];
    __imag__ z = im.empty() ? 0 : (__float128)im[j];
    E[(e - 1) / 2] = z;
    cq zc;
    __real__ zc = __real__ z;
    __imag__ zc = -__imag__ z;
    E[(twoN - e - 1) / 2] = zc;
    e = (e * 5) % twoN;
  }
  return E;
}

std::vector<i64> encode_int(const Context& C, const std::vector<double>& re,
                            const std::vector<double>& im, double scale) {
  std::vector<cq> E = slots_to_evals(C, re, im);
  fft_q(E, -1);   // F_i = sum_t E_t omega^{-t i}
  std::vector<i64> m(C.N);
  for (int i = 0; i < C.N; i++) {
    cq tw = expi(-M_PIq * (__float128)i / (__float128)C.N);   // zeta^{-i}
    cq v = E[i] * tw;
    m[i] = round_half_away((__float128)scale * __real__ v / (__float128)C.N);
  }
  return m;
}

std::vector<i64> encode_int_direct(const Context& C, const std::vector<double>& re,
                                   const std::vector<double>& im, double scale) {
  std::vector<cq> E = slots_to_evals(C, re, im);
  std::vector<i64> m(C.N);
  for (int i = 0; i < C.N; i++) {
    cq acc = 0;
    for (int t = 0; t < C.N; t++) {
      u64 ex = ((2 * (u64)t + 1) * (u64)i) % (2 * (u64)C.N);
      acc += E[t] * expi(-M_PIq * (__float128)ex / (__float128)C.N);
    }
    m[i] = round_half_away((__float128)scale * __real__ acc / (__float128)C.N);
  }
  return m;
}

RPoly encode(const Context& C, const std::vector<double>& re, const std::vector<double>& im,
             double scale, const std::vector<int>& pidx) {
  std::vector<i64> m = encode_int(C, re, im, scale);
  RPoly r = poly_zero(C, pidx);
  for (size_t l = 0; l < pidx.size(); l++)
    for (int i = 0; i < C.N; i++) r.c[l][i] = from_i64(m[i], C.primes[pidx[l]]);
  return r;
}

void decode(const Context& C, const Vec& limb0, u64 q0, double scale, std::vector<double>& re,
            std::vector<double>& im) {
  std::vector<cq> a(C.N);
  for (int i = 0; i < C.N; i++) {
    i64 v = limb0[i] <= (q0 - 1) / 2 ? (i64)limb0[i] : (i64)limb0[i] - (i64)q0;
    a[i] = (__float128)v * expi(M_PIq * (__float128)i / (__float128)C.N);   // m_i zeta^i
  }
  fft_q(a, +1);   // E_t = sum_i m_i zeta^i omega^{t i} = m(zeta^{2t+1})
  re.assign(C.ns, 0);
  im.assign(C.ns, 0);
  u64 e = 1;
  const u64 twoN = 2 * (u64)C.N;
  for (int j = 0; j < C.ns; j++) {
    cq z = a[(e - 1) / 2];
    re[j] = (double)(__real__ z / (__float128)scale);
    im[j] = (double)(__imag__ z / (__float128)scale);
    e = (e * 5) % twoN;
  }
}

}  // namespace orc
