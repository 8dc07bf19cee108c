// Peak-rate microbenchmarks for gfx950 (a measuring tool beside the library,
// not part of the evaluation path).
//
// Instruction issue rates: each thread runs C independent dependency chains of
// one operation, so the rate reflects issue throughput rather than latency.
// Modular-multiply rates on a 50-bit modulus compare the library's binary64
// forms (fenc_arith.h, unchanged) with 64-bit integer forms built from 32-bit
// multiplies: Shoup for a constant operand, Montgomery and Barrett for two
// variable operands.  Every modular chain computes x0 * w^iters mod q; the host
// checks a sample of chains against 128-bit integer arithmetic.  HBM ceilings:
// copy, read-only and write-only kernels with 16-byte accesses over
// multi-GiB buffers, and the runtime's device-to-device copy.
//
// C ABI (results are per call; timing is the best of several launches):
//   int         fenc_peaks_count(void);
//   const char* fenc_peaks_name(int i);   // "name|unit"
//   int         fenc_peaks_run(int i, double bytes_or_target_s,
//                              double* seconds, double* work, int* exact);
// For instruction and modular tests the second argument is the target
// duration of one launch in seconds; for memory tests it is the buffer size
// in bytes.  work is the count the unit refers to (operations, flops or
// bytes); exact is 1 when the host check passed, 0 when it failed and -1
// where there is nothing to check.  Returns 0, or -1 on a HIP error.
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#define FENC_HD __host__ __device__
#include "fenc_arith.h"

namespace {

constexpr int kThreads = 256;
constexpr int kBlocks = 2048;   // 8 blocks of 4 waves on each of 256 CUs
constexpr int kChains = 8;
constexpr int kLanes = kThreads * kBlocks;
typedef unsigned long long u64;

// ---------------------------------------------------------------- issue rates
__global__ __launch_bounds__(kThreads) void k_fma(double* out, double y, double z, int iters) {
  const int t = blockIdx.x * kThreads + threadIdx.x;
  double x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = t * 1e-9 + c;
#pragma unroll 4
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = fma(x[c], y, z);
  }
  double s = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += x[c];
  out[t] = s;
}

__global__ __launch_bounds__(kThreads) void k_mulhi(unsigned* out, unsigned m, int iters) {
  const unsigned t = blockIdx.x * kThreads + threadIdx.x;
  unsigned x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = t * 2654435761u + c;
#pragma unroll 4
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = __umulhi(x[c], m);
  }
  unsigned s = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s ^= x[c];
  out[t] = s;
}

__global__ __launch_bounds__(kThreads) void k_mullo(unsigned* out, unsigned m, int iters) {
  const unsigned t = blockIdx.x * kThreads + threadIdx.x;
  unsigned x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = (t * 2654435761u + 2 * c) | 1u;
  // squaring keeps odd values odd and cannot be reassociated into fewer steps
#pragma unroll 4
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = x[c] * x[c];
  }
  x[0] ^= m;
  unsigned s = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s ^= x[c];
  out[t] = s;
}

// acc <- hi32(acc) * m + k: one 32x32+64 multiply-add per step (the high half
// feeds the next step, so no step can be done in 32-bit pieces)
__global__ __launch_bounds__(kThreads) void k_mad64(u64* out, unsigned m, u64 k, int iters) {
  const unsigned t = blockIdx.x * kThreads + threadIdx.x;
  u64 x[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) x[c] = (u64)t * 0x9E3779B97F4A7C15ull + c;
#pragma unroll 4
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = (u64)(unsigned)(x[c] >> 32) * m + k;
  }
  u64 s = 0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s ^= x[c];
  out[t] = s;
}

// ----------------------------------------------------------- modular multiply
struct ModArgs {
  u64 q, w;          // modulus and multiplier
  double qd, qinv, wd, wq;
  u64 wp;            // floor(w 2^64 / q)       (Shoup)
  u64 wr, qneg;      // w 2^64 mod q, -q^-1 mod 2^64   (Montgomery)
  u64 mu;            // floor(2^100 / q)        (Barrett, 2^49 < q < 2^50)
};

__host__ __device__ inline u64 chain_start(unsigned t, int c) { return (u64)(t * kChains + c) * 1000003ull + 17; }

__device__ inline u64 shoup(u64 x, u64 w, u64 wp, u64 q) {
  const u64 r = x * w - __umul64hi(x, wp) * q;   // in [0, 2q)
  return r >= q ? r - q : r;
}

__device__ inline u64 montgomery(u64 a, u64 b, u64 q, u64 qneg) {
  const u64 lo = a * b, hi = __umul64hi(a, b);
  const u64 m = lo * qneg;                       // lo + m q = 0 mod 2^64
  const u64 t = hi + __umul64hi(m, q) + (lo != 0);
  return t >= q ? t - q : t;
}

__device__ inline u64 barrett50(u64 a, u64 b, u64 q, u64 mu) {
  const u64 lo = a * b, hi = __umul64hi(a, b);   // a b < 2^100
  const u64 x = (hi << 15) | (lo >> 49);         // floor(a b / 2^49) < 2^51
  const u64 qh = (__umul64hi(x, mu) << 13) | ((x * mu) >> 51);
  u64 r = lo - qh * q;                           // in [0, 3q)
  r = r >= q ? r - q : r;
  return r >= q ? r - q : r;
}

template <int V>
__global__ __launch_bounds__(kThreads) void k_mod(u64* out, ModArgs a, int iters) {
  const unsigned t = blockIdx.x * kThreads + threadIdx.x;
  if constexpr (V <= 1) {
    double x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = (double)chain_start(t, c);
#pragma unroll 4
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int c = 0; c < kChains; ++c)
        x[c] = V == 0 ? fk::mulmod(x[c], a.wd, a.qd, a.qinv) : fk::mulmod_c(x[c], a.wd, a.wq, a.qd);
    }
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      double r = x[c] < 0 ? x[c] + a.qd : x[c];
      out[(size_t)t * kChains + c] = (u64)(r >= a.qd ? r - a.qd : r);
    }
  } else {
    u64 x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = chain_start(t, c);
#pragma unroll 4
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int c = 0; c < kChains; ++c)
        x[c] = V == 2 ? shoup(x[c], a.w, a.wp, a.q)
             : V == 3 ? montgomery(x[c], a.wr, a.q, a.qneg)
                      : barrett50(x[c], a.w, a.q, a.mu);
    }
#pragma unroll
    for (int c = 0; c < kChains; ++c) out[(size_t)t * kChains + c] = x[c];
  }
}

// ------------------------------------------------------------------- memory
__global__ __launch_bounds__(kThreads) void k_copy(const uint4* __restrict__ s, uint4* __restrict__ d, size_t n) {
  const size_t stride = (size_t)gridDim.x * kThreads;
  size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const uint4 a = s[i], b = s[i + stride], c = s[i + 2 * stride], e = s[i + 3 * stride];
    d[i] = a; d[i + stride] = b; d[i + 2 * stride] = c; d[i + 3 * stride] = e;
  }
  for (; i < n; i += stride) d[i] = s[i];
}

__global__ __launch_bounds__(kThreads) void k_read(const uint4* __restrict__ s, unsigned* out, size_t n) {
  const size_t stride = (size_t)gridDim.x * kThreads;
  size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x;
  unsigned acc = 0;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const uint4 a = s[i], b = s[i + stride], c = s[i + 2 * stride], e = s[i + 3 * stride];
    acc ^= a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w ^ c.x ^ c.y ^ c.z ^ c.w ^ e.x ^ e.y ^ e.z ^ e.w;
  }
  for (; i < n; i += stride) acc ^= s[i].x ^ s[i].w;
  out[(size_t)blockIdx.x * kThreads + threadIdx.x] = acc;
}

__global__ __launch_bounds__(kThreads) void k_write(uint4* __restrict__ d, size_t n) {
  const size_t stride = (size_t)gridDim.x * kThreads;
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride)
    d[i] = make_uint4((unsigned)i, (unsigned)(i >> 32), 1u, 2u);
}

// ------------------------------------------------------------------- host side
const char* kNames[] = {
    "fp64 FMA (v_fma_f64)|flop",
    "32-bit multiply high (v_mul_hi_u32)|op",
    "32-bit multiply low (v_mul_lo_u32)|op",
    "32x32+64 multiply-add (v_mad_u64_u32)|op",
    "binary64 mulmod, both operands variable|modmul",
    "binary64 mulmod_c, constant operand with w/q|modmul",
    "u64 Shoup, constant operand with floor(w 2^64/q)|modmul",
    "u64 Montgomery, both operands variable|modmul",
    "u64 Barrett, both operands variable|modmul",
    "copy kernel, 16 B per lane (read + write)|byte",
    "read kernel, 16 B per lane|byte",
    "write kernel, 16 B per lane|byte",
    "hipMemcpyAsync device to device (read + write)|byte",
};
constexpr int kCount = sizeof(kNames) / sizeof(kNames[0]);

// Best of `reps` timed launches in seconds, or -1 when a HIP call fails.
template <class L>
double best_seconds(L launch, int reps) {
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return -1;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return -1;
  }
  bool ok = true;
  launch();   // warm-up
  float best = 1e30f;
  for (int r = 0; r < reps && ok; ++r) {
    float ms = 0;
    ok = hipEventRecord(a, 0) == hipSuccess;
    launch();
    ok = ok && hipGetLastError() == hipSuccess && hipEventRecord(b, 0) == hipSuccess &&
         hipEventSynchronize(b) == hipSuccess && hipEventElapsedTime(&ms, a, b) == hipSuccess;
    if (ok && ms < best) best = ms;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return ok ? best * 1e-3 : -1;
}

// iteration count giving about target seconds per launch
template <class F>
int calibrate(F run_iters, double target) {
  const int base = 256;
  const double t = run_iters(base);
  if (t <= 0) return -1;
  double k = target / t * base;
  if (k < base) k = base;
  if (k > (1 << 24)) k = 1 << 24;
  return (int)k;
}

u64 powmod(u64 x, u64 w, u64 e, u64 q) {
  unsigned __int128 r = x % q, b = w % q;
  while (e) {
    if (e & 1) r = r * b % q;
    b = b * b % q;
    e >>= 1;
  }
  return (u64)r;
}

ModArgs mod_args() {
  ModArgs a;
  a.q = 1125899906842597ull;         // 2^50 - 27 (odd, in (2^49, 2^50))
  a.w = 876543210987654ull % a.q;
  a.qd = (double)a.q;
  a.qinv = 1.0 / a.qd;
  a.wd = (double)a.w;
  a.wq = a.wd / a.qd;
  a.wp = (u64)(((unsigned __int128)a.w << 64) / a.q);
  a.wr = (u64)(((unsigned __int128)a.w << 64) % a.q);
  u64 inv = 1;   // q^-1 mod 2^64 by Newton iteration
  for (int i = 0; i < 6; ++i) inv *= 2 - a.q * inv;
  a.qneg = 0 - inv;
  a.mu = (u64)(((unsigned __int128)1 << 100) / a.q);
  return a;
}

}  // namespace

extern "C" int fenc_peaks_count(void) { return kCount; }

extern "C" const char* fenc_peaks_name(int i) { return i >= 0 && i < kCount ? kNames[i] : nullptr; }

extern "C" int fenc_peaks_run(int test, double arg, double* seconds, double* work, int* exact) {
  if (test < 0 || test >= kCount) return -1;
  *exact = -1;
  const dim3 grid(kBlocks), block(kThreads);
  if (test <= 8) {
    void* out = nullptr;
    if (hipMalloc(&out, (size_t)kLanes * kChains * sizeof(u64)) != hipSuccess) return -1;
    const ModArgs ma = mod_args();
    auto launch = [&](int iters) {
      switch (test) {
        case 0: hipLaunchKernelGGL(k_fma, grid, block, 0, 0, (double*)out, 0.999999, 1e-3, iters); break;
        case 1: hipLaunchKernelGGL(k_mulhi, grid, block, 0, 0, (unsigned*)out, 0x9E3779B9u, iters); break;
        case 2: hipLaunchKernelGGL(k_mullo, grid, block, 0, 0, (unsigned*)out, 0x9E3779B9u, iters); break;
        case 3: hipLaunchKernelGGL(k_mad64, grid, block, 0, 0, (u64*)out, 0x9E3779B9u, 12345ull, iters); break;
        case 4: hipLaunchKernelGGL(k_mod<0>, grid, block, 0, 0, (u64*)out, ma, iters); break;
        case 5: hipLaunchKernelGGL(k_mod<1>, grid, block, 0, 0, (u64*)out, ma, iters); break;
        case 6: hipLaunchKernelGGL(k_mod<2>, grid, block, 0, 0, (u64*)out, ma, iters); break;
        case 7: hipLaunchKernelGGL(k_mod<3>, grid, block, 0, 0, (u64*)out, ma, iters); break;
        default: hipLaunchKernelGGL(k_mod<4>, grid, block, 0, 0, (u64*)out, ma, iters); break;
      }
    };
    const int iters = calibrate([&](int it) { return best_seconds([&] { launch(it); }, 2); }, arg);
    if (iters < 0) {
      (void)hipFree(out);
      return -1;
    }
    *seconds = best_seconds([&] { launch(iters); }, 5);
    *work = (double)kLanes * kChains * iters * (test == 0 ? 2.0 : 1.0);
    if (test >= 4) {
      std::vector<u64> h((size_t)kLanes * kChains);
      if (hipMemcpy(h.data(), out, h.size() * sizeof(u64), hipMemcpyDeviceToHost) != hipSuccess) {
        (void)hipFree(out);
        return -1;
      }
      int ok = 1;
      for (unsigned t = 0; t < (unsigned)kLanes; t += 97)
        for (int c = 0; c < kChains; ++c)
          if (h[(size_t)t * kChains + c] != powmod(chain_start(t, c), ma.w, iters, ma.q)) ok = 0;
      *exact = ok;
    }
    (void)hipFree(out);
    return *seconds > 0 ? 0 : -1;
  }
  const size_t bytes = (size_t)arg & ~(size_t)4095;
  const size_t n = bytes / sizeof(uint4);
  void *s = nullptr, *d = nullptr;
  auto release = [&] {
    (void)hipFree(s);
    if (d) (void)hipFree(d);
  };
  if (hipMalloc(&s, bytes) != hipSuccess) return -1;
  if ((test != 10 && test != 11 && hipMalloc(&d, bytes) != hipSuccess) ||
      (test == 10 && hipMalloc(&d, (size_t)kLanes * 4 * sizeof(unsigned)) != hipSuccess) ||
      hipMemset(s, 1, bytes) != hipSuccess) {
    release();
    return -1;
  }
  const dim3 mgrid(kBlocks * 2);
  bool copy_failed = false;
  auto launch = [&] {
    switch (test) {
      case 9: hipLaunchKernelGGL(k_copy, mgrid, block, 0, 0, (const uint4*)s, (uint4*)d, n); break;
      case 10: hipLaunchKernelGGL(k_read, mgrid, block, 0, 0, (const uint4*)s, (unsigned*)d, n); break;
      case 11: hipLaunchKernelGGL(k_write, mgrid, block, 0, 0, (uint4*)s, n); break;
      default:
        if (hipMemcpyAsync(d, s, bytes, hipMemcpyDeviceToDevice, 0) != hipSuccess) copy_failed = true;
        break;
    }
  };
  *seconds = best_seconds(launch, 5);
  if (copy_failed) *seconds = -1;
  *work = (double)bytes * (test == 9 || test == 12 ? 2.0 : 1.0);
  if (test == 9 || test == 12) {   // the copy arrived: compare a few words
    unsigned char a[4096], b[4096];
    if (hipMemcpy(a, (char*)s + bytes - 4096, 4096, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(b, (char*)d + bytes - 4096, 4096, hipMemcpyDeviceToHost) != hipSuccess)
      *exact = 0;
    else
      *exact = memcmp(a, b, 4096) == 0;
  }
  release();
  return *seconds > 0 ? 0 : -1;
}
