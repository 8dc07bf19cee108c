// Kernel bodies of the hot path.
//
// Each body is written against a small execution interface X:
//   x.bx, x.by, x.bz   block indices
//   x.nt               threads per block
//   x.smem             LDS scratch (doubles)
//   x.phase(f)         run f(tid) for the threads of the block, then barrier
// The HIP backend instantiates X as "this thread"; the test suite also runs
// the same bodies through a sequential emulator to check index arithmetic on
// the CPU.  Residues are uint64 in [0, q) in HBM and exact integers in
// binary64 inside the kernels (fenc_arith.h).
#pragma once
#include <cstddef>
#include <type_traits>
#include "fenc_arith.h"

namespace fk {

struct d2 {
  double x, y;
};

#ifndef FENC_AI
#define FENC_AI __attribute__((always_inline)) inline
#endif
#ifndef FENC_GLOBAL
#define FENC_GLOBAL
#endif
// Loads and stores through device pointers known to address global memory;
// w2: two adjacent words, 16-byte aligned.
typedef u64 w2 __attribute__((vector_size(16)));
FENC_HD FENC_AI u64 ldg(const u64* p) { return *(const FENC_GLOBAL u64*)p; }
FENC_HD FENC_AI w2 ldg2(const u64* p) { return *(const FENC_GLOBAL w2*)p; }
FENC_HD FENC_AI void stg2(u64* p, u64 x, u64 y) {
  w2 v;
  v[0] = x;
  v[1] = y;
  *(FENC_GLOBAL w2*)p = v;
}

constexpr int kMaxMap = 128;
constexpr unsigned char kSkip = 255;

// prime of row r is p[r % n]; kSkip leaves the row untouched
struct PrimeMap {
  int n;
  unsigned char p[kMaxMap];
};

// ------------------------------------------------------------------ XCD-aware block order
// The chip dispatches the blocks of a launch round-robin over its 8 XCDs
// (block p runs on XCD p % 8), and each XCD has its own L2.  A launch made
// with this order runs as a 1-D grid of gx*gy*gz blocks; every XCD receives a
// contiguous range of the logical order in which z varies fastest, so blocks
// that differ only in z (and read the same tile of a shared operand) run on
// one XCD, close in time.
constexpr unsigned kXcds = 8;
FENC_HD inline void xcd_coords(unsigned p, unsigned gx, unsigned gy, unsigned gz, int& bx, int& by, int& bz) {
  const unsigned nb = gx * gy * gz, q = nb / kXcds, rem = nb % kXcds, r = p % kXcds;
  const unsigned L = r * q + (r < rem ? r : rem) + p / kXcds;
  bz = (int)(L % gz);
  const unsigned rest = L / gz;
  bx = (int)(rest % gx);
  by = (int)(rest / gx);
}

// ------------------------------------------------------------------ NTT
// Negacyclic NTT over rows of N = 2^logn residues.  Forward: Cooley-Tukey
// with merged psi twiddles, natural order in, bit-reversed order out (slot k
// holds the evaluation at psi^(2 brev(k)+1)).  Inverse: Gentleman-Sande,
// bit-reversed in, natural out, scaled by N^-1.  Split into a column pass
// (stride-2^n2 butterflies, first n1 forward stages) and a row pass
// (contiguous chunks of 2^n2, last n2 stages); both stage their tile in LDS.
struct NttArgs {
  const u64* src;
  u64* dst;
  long long src_gs, dst_gs;   // elements between row groups
  int nrows, nl;              // rows, rows per group (row r: group r/nl, limb r%nl)
  PrimeMap pm;
  const double* tw;           // [prime][N] twiddles w; the quotient estimate w/q is formed as w * (1/q)
  const d2* pq;               // [prime] (q, 1/q)
  const d2* ninv;             // [prime] (N^-1, N^-1/q), inverse only
  int logn, n1, n2;
  int lcols;                  // log2 of the columns per block (column pass)
  int lcpb;                   // log2 of the chunks per block (row pass)
};


// Twiddle pair (w, w/q) for mulmod_c from w alone; the twiddle table holds 8
// bytes per entry.  The estimate fl(w * fl(1/q)) has relative error below
// 2^-52, so for q < 2^50 mulmod_c keeps its contract (fenc_arith.h): the
// exact a*w - e*q for a*w/q > -2^51, of magnitude at most (1/2 + |a|/(4q)) q
// while a*w/q < 2^51 and (1 + |a|/(4q)) q above.
FENC_HD inline d2 twiddle(double w, double qi) { return d2{w, w * qi}; }

// Stage index of member f (< 2^k) of the butterfly group whose other stage
// bits are `rest`, with the k-bit field at bit `lo`.
FENC_HD inline int member(int rest, int f, int lo, int k) {
  return ((((rest >> lo) << k) | f) << lo) | (rest & ((1 << lo) - 1));
}

// One register round of forward (Cooley-Tukey) stages s0..s0+K-1 of a pass
// with P stage bits: local stage s pairs stage-index bit P-1-s.  tw_of(s, a)
// is the twiddle of the butterfly whose upper element has stage index a.
// Inputs come from HBM in [0, q) or from LDS reduced to [-q/2 - 1, q/2 + 1];
// outputs are reduced to [-q/2, q/2] (up to one unit).  Operand ranges of
// the products (the multiplicand a of mulmod_c, w < q):
//   HBM inputs:  stage 1 a in [0, q), sums in [-0.75q, 1.75q); stage 2 a in
//                that range, sums in [-1.69q, 2.69q]; stage 3 a in that range:
//                a*w/q >= -1.69 * 2^50 > -2^51 (exact), above 2^51 the
//                estimate rounds to even, |t| <= 1.68q, sums within 4.37q;
//   LDS inputs:  sums within 1.13q and 1.91q; stage 3 a*w/q >= -1.91 * 2^50.
// Every sum stays below 2^53 and exact.  A fourth stage (K = 4) follows a
// reduction, so its inputs are LDS-like.  K is a compile-time constant so the
// group lives in registers.
template <int K, class LD, class ST, class TW>
FENC_HD inline void fwd_round(int rest, int s0, int P, double q, double qi, LD ld, ST st, TW tw_of) {
  double v[1 << K];
  const int lo = P - s0 - K;
#pragma unroll
  for (int f = 0; f < (1 << K); f++) v[f] = ld(member(rest, f, lo, K));
#pragma unroll
  for (int s = 0; s < K; s++) {
    if (s == 3) {   // K = 4: bring the values back below q/2 before the fourth stage
#pragma unroll
      for (int f = 0; f < (1 << K); f++) v[f] = red(v[f], q, qi);
    }
    const int half = 1 << (K - 1 - s);
#pragma unroll
    for (int f = 0; f < (1 << K); f++) {
      if (f & half) continue;
      const d2 w = tw_of(s0 + s, member(rest, f, lo, K));
      const double u = v[f], t = mulmod_c(v[f | half], w.x, w.y, q);
      v[f] = u + t;
      v[f | half] = u - t;
    }
  }
#pragma unroll
  for (int f = 0; f < (1 << K); f++) st(member(rest, f, lo, K), red(v[f], q, qi));
}

// One register round of inverse (Gentleman-Sande) stages s0..s0+K-1: local
// stage s pairs stage-index bit s.  Inputs and outputs have magnitude < q:
// the difference x - y lies within 2q, so |a*w/q| < 2^51 and the product is
// at most (1/2 + 2q/(4q)) q < q; the sum is reduced.
template <int K, class LD, class ST, class TW>
FENC_HD inline void inv_round(int rest, int s0, double q, double qi, LD ld, ST st, TW tw_of) {
  double v[1 << K];
  const int lo = s0;
#pragma unroll
  for (int f = 0; f < (1 << K); f++) v[f] = ld(member(rest, f, lo, K));
#pragma unroll
  for (int s = 0; s < K; s++) {
    const int half = 1 << s;
#pragma unroll
    for (int f = 0; f < (1 << K); f++) {
      if (f & half) continue;
      const d2 w = tw_of(s0 + s, member(rest, f, lo, K));
      const double xv = v[f], yv = v[f | half];
      v[f] = red(xv + yv, q, qi);
      v[f | half] = mulmod_c(xv - yv, w.x, w.y, q);
    }
  }
#pragma unroll
  for (int f = 0; f < (1 << K); f++) st(member(rest, f, lo, K), v[f]);
}

// Round schedule of a pass with P stage bits and rounds of at most RB stages:
// ceil(P/RB) register rounds of nearly equal size (larger rounds first).
FENC_HD constexpr int n_rounds(int P, int RB) { return (P + RB - 1) / RB; }
FENC_HD constexpr int round_size(int P, int RB, int r) {
  return P / n_rounds(P, RB) + (r < P % n_rounds(P, RB) ? 1 : 0);
}
FENC_HD constexpr int round_start(int P, int RB, int r) {
  return r == 0 ? 0 : round_start(P, RB, r - 1) + round_size(P, RB, r - 1);
}

template <int R, int NR>
struct RoundLoop {
  template <class B>
  FENC_HD static void run(B body) {
    body(std::integral_constant<int, R>());
    RoundLoop<R + 1, NR>::run(body);
  }
};
template <int NR>
struct RoundLoop<NR, NR> {
  template <class B>
  FENC_HD static void run(B) {}
};

// Calls body(integral_constant<P>) for the pass size p in 1..8.
template <class B>
FENC_HD inline void with_pass(int p, B body) {
  switch (p) {
    case 1: body(std::integral_constant<int, 1>()); break;
    case 2: body(std::integral_constant<int, 2>()); break;
    case 3: body(std::integral_constant<int, 3>()); break;
    case 4: body(std::integral_constant<int, 4>()); break;
    case 5: body(std::integral_constant<int, 5>()); break;
    case 6: body(std::integral_constant<int, 6>()); break;
    case 7: body(std::integral_constant<int, 7>()); break;
    default: body(std::integral_constant<int, 8>()); break;
  }
}

// Calls body(integral_constant<n>) for a small count n in 1..8, else with 16
// (the body then guards with the runtime count).
template <class B>
FENC_HD inline void with_count(int n, B body) {
  switch (n) {
    case 1: body(std::integral_constant<int, 1>()); break;
    case 2: body(std::integral_constant<int, 2>()); break;
    case 3: body(std::integral_constant<int, 3>()); break;
    case 4: body(std::integral_constant<int, 4>()); break;
    case 5: body(std::integral_constant<int, 5>()); break;
    case 6: body(std::integral_constant<int, 6>()); break;
    case 7: body(std::integral_constant<int, 7>()); break;
    case 8: body(std::integral_constant<int, 8>()); break;
    default: body(std::integral_constant<int, 16>()); break;
  }
}

struct NoPro {};

// Column pass: stages acting on 2^n1 elements at stride 2^n2 ("columns").  A
// block stages 2^lcols adjacent columns; the column index is the low part of
// the thread's group index so neighbouring threads touch neighbouring words.
// Forward: the first n1 stages; inverse: the last n1 stages, then * N^-1.
// The first round reads HBM, the last writes HBM, the others use LDS.
// With a prologue (PRO other than NoPro) the first round takes each input
// value from pro_load(row, element) (magnitude < q) instead of reading src.
template <bool INV, int P, int RB, class PRO = NoPro, class X>
FENC_HD void ntt_cols_pass(X& x, const NttArgs& a, int p, const PRO* pro = nullptr) {
  const int n2 = a.n2, sb = a.lcols, T = x.nt, bm = (1 << sb) - 1;
  const int row = x.by;
  const u64* src = a.src + (long long)(row / a.nl) * a.src_gs + ((long long)(row % a.nl) << a.logn);
  u64* dst = a.dst + (long long)(row / a.nl) * a.dst_gs + ((long long)(row % a.nl) << a.logn);
  const long long col0 = (long long)x.bx << sb;
  const double q = a.pq[p].x, qi = a.pq[p].y;
  const double* tw = a.tw + ((long long)p << a.logn);
  double* sm = x.smem;
  const d2 ni = INV ? a.ninv[p] : d2{0, 0};
  // the pass uses the 2^P twiddles tw[0, 2^P) of every column: staged once in
  // LDS after the tile, so the rounds read them there
  double* twl = sm + (1 << (P + sb));
  x.phase([&](int t) {
    for (int i = t; i < (1 << P); i += T) twl[i] = tw[i];
  });
  RoundLoop<0, n_rounds(P, RB)>::run([&](auto R) {
    constexpr int r = decltype(R)::value;
    constexpr int K = round_size(P, RB, r), s0 = round_start(P, RB, r);
    constexpr bool first = r == 0, last = r == n_rounds(P, RB) - 1;
    x.phase([&](int t) {
      for (int g = t; g < (1 << (P + sb - K)); g += T) {
        const int c = g & bm, rest = g >> sb;
        auto ld = [&](int hi) {
          if constexpr (!std::is_same<PRO, NoPro>::value) {
            if (first) return pro_load(*pro, row, ((long long)hi << n2) + col0 + c, q, qi);
          } else {
            if (first) return u2d(src[((long long)hi << n2) + col0 + c]);
          }
          return sm[(hi << sb) | c];
        };
        if constexpr (!INV) {
          fwd_round<K>(
              rest, s0, P, q, qi, ld,
              [&](int hi, double v) {
                if (last) dst[((long long)hi << n2) + col0 + c] = d2u(norm(v, q));
                else sm[(hi << sb) | c] = v;
              },
              [&](int st, int hi) { return twiddle(twl[(1 << st) + (hi >> (P - st))], qi); });
        } else {
          inv_round<K>(
              rest, s0, q, qi, ld,
              [&](int hi, double v) {
                if (last) dst[((long long)hi << n2) + col0 + c] = d2u(norm(mulmod_c(v, ni.x, ni.y, q), q));
                else sm[(hi << sb) | c] = v;
              },
              // global stage u = n2 + st: h = N >> (u+1), group = hi >> (st+1)
              [&](int st, int hi) { return twiddle(twl[(1 << (P - st - 1)) + (hi >> (st + 1))], qi); });
        }
      }
    });
  });
}

// Row pass: stages acting inside contiguous chunks of 2^n2 elements; a block
// stages 2^lcpb chunks.  The chunk is the high part of the thread's group
// index so neighbouring threads touch neighbouring words.  Forward: the last
// n2 stages; inverse: the first n2 stages.
// The last forward round writes its groups at a stride of 2^K words; it
// writes the LDS tile instead, and the block's words, which are contiguous,
// go to HBM in a separate coalesced phase.  (Staging the strided first round
// of the inverse pass the same way was measured slower.)  With an epilogue
// (EPI other than NoEpi) that phase hands each value (row, element, v in
// [-q/2, q/2]) to the epilogue instead of writing dst: epi_load fetches the
// epilogue's own input words for an element, epi_finish computes and stores
// its output.
struct NoEpi {};
constexpr int kEpiBatch = 4;   // elements whose epilogue loads are issued together

template <bool INV, int P, int RB, class EPI = NoEpi, class X>
FENC_HD void ntt_rows_pass(X& x, const NttArgs& a, int p, const EPI* epi = nullptr) {
  constexpr bool plain = std::is_same<EPI, NoEpi>::value;
  constexpr bool stage_out = !INV;
  const int n1 = a.n1, cb = a.lcpb, T = x.nt, logn = a.logn;
  const int row = x.by;
  const long long e0 = (long long)x.bx << (P + cb);
  const u64* src = a.src + (long long)(row / a.nl) * a.src_gs + ((long long)(row % a.nl) << logn) + e0;
  u64* dst = a.dst + (long long)(row / a.nl) * a.dst_gs + ((long long)(row % a.nl) << logn) + e0;
  const long long chunk0 = (long long)x.bx << cb;
  const double q = a.pq[p].x, qi = a.pq[p].y;
  const double* tw = a.tw + ((long long)p << logn);
  double* sm = x.smem;
  RoundLoop<0, n_rounds(P, RB)>::run([&](auto R) {
    constexpr int r = decltype(R)::value;
    constexpr int K = round_size(P, RB, r), s0 = round_start(P, RB, r);
    constexpr bool first = r == 0, last = r == n_rounds(P, RB) - 1;
    x.phase([&](int t) {
      for (int g = t; g < (1 << (P + cb - K)); g += T) {
        const int rest = g & ((1 << (P - K)) - 1), ch = g >> (P - K);
        const int base = ch << P;
        auto ld = [&](int lo) { return first ? u2d(src[base + lo]) : sm[base + lo]; };
        auto st = [&](int lo, double v) {
          if (last && !stage_out) dst[base + lo] = d2u(norm(v, q));
          else sm[base + lo] = v;
        };
        if constexpr (!INV) {
          fwd_round<K>(rest, s0, P, q, qi, ld, st,
                       // global stage n1 + st: group = (chunk << st) + (lo >> (n2 - st))
                       [&](int s, int lo) {
                         return twiddle(tw[(1LL << (n1 + s)) + ((chunk0 + ch) << s) + (lo >> (P - s))], qi);
                       });
        } else {
          inv_round<K>(rest, s0, q, qi, ld, st,
                       // stage s: h = N >> (s+1), group = (chunk << (n2-s-1)) + (lo >> (s+1))
                       [&](int s, int lo) {
                         return twiddle(tw[(1LL << (logn - s - 1)) + ((chunk0 + ch) << (P - s - 1)) + (lo >> (s + 1))], qi);
                       });
        }
      }
    });
  });
  if constexpr (stage_out) {
    x.phase([&](int t) {
      const int n = 1 << (P + cb);
      if constexpr (plain) {
        for (int g = t; g < n; g += T) dst[g] = d2u(norm(sm[g], q));
      } else {
        // the epilogue's loads of kEpiBatch words are issued before any of
        // their stores (a store may alias them as far as the compiler knows);
        // slots past the tile reload word g0, which exists, and store nothing
        for (int g0 = t; g0 < n; g0 += kEpiBatch * T) {
          decltype(epi_load(*epi, row, e0, q, qi)) pre[kEpiBatch];
#pragma unroll
          for (int j = 0; j < kEpiBatch; j++) {
            const int g = g0 + j * T;
            pre[j] = epi_load(*epi, row, e0 + (g < n ? g : g0), q, qi);
          }
#pragma unroll
          for (int j = 0; j < kEpiBatch; j++) {
            const int g = g0 + j * T;
            if (g < n) epi_finish(*epi, row, e0 + g, pre[j], sm[g], q, qi);
          }
        }
      }
    });
  }
}

// Kernel entries: radix-8 rounds (RB = 3) and radix-16 rounds (RB = 4).
template <int RB, class X>
FENC_HD void ntt_fwd_cols_rb(X& x, const NttArgs& a) {
  const int p = a.pm.p[x.by % a.pm.n];
  if (p == kSkip) return;
  with_pass(a.n1, [&](auto P) { ntt_cols_pass<false, decltype(P)::value, RB>(x, a, p); });
}
template <int RB, class X>
FENC_HD void ntt_inv_cols_rb(X& x, const NttArgs& a) {
  const int p = a.pm.p[x.by % a.pm.n];
  if (p == kSkip) return;
  with_pass(a.n1, [&](auto P) { ntt_cols_pass<true, decltype(P)::value, RB>(x, a, p); });
}
template <int RB, class X>
FENC_HD void ntt_fwd_rows_rb(X& x, const NttArgs& a) {
  const int p = a.pm.p[x.by % a.pm.n];
  if (p == kSkip) return;
  with_pass(a.n2, [&](auto P) { ntt_rows_pass<false, decltype(P)::value, RB>(x, a, p); });
}
template <int RB, class X>
FENC_HD void ntt_inv_rows_rb(X& x, const NttArgs& a) {
  const int p = a.pm.p[x.by % a.pm.n];
  if (p == kSkip) return;
  with_pass(a.n2, [&](auto P) { ntt_rows_pass<true, decltype(P)::value, RB>(x, a, p); });
}
template <class X> FENC_HD void ntt_fwd_cols(X& x, const NttArgs& a) { ntt_fwd_cols_rb<3>(x, a); }
template <class X> FENC_HD void ntt_inv_cols(X& x, const NttArgs& a) { ntt_inv_cols_rb<3>(x, a); }
template <class X> FENC_HD void ntt_fwd_rows(X& x, const NttArgs& a) { ntt_fwd_rows_rb<3>(x, a); }
template <class X> FENC_HD void ntt_inv_rows(X& x, const NttArgs& a) { ntt_inv_rows_rb<3>(x, a); }
template <class X> FENC_HD void ntt_fwd_cols16(X& x, const NttArgs& a) { ntt_fwd_cols_rb<4>(x, a); }
template <class X> FENC_HD void ntt_inv_cols16(X& x, const NttArgs& a) { ntt_inv_cols_rb<4>(x, a); }
template <class X> FENC_HD void ntt_fwd_rows16(X& x, const NttArgs& a) { ntt_fwd_rows_rb<4>(x, a); }
template <class X> FENC_HD void ntt_inv_rows16(X& x, const NttArgs& a) { ntt_inv_rows_rb<4>(x, a); }

// ------------------------------------------------------------------ ModUp
// Fast base conversion of every digit of c1 (coefficient form) to the other
// limbs of Q_l U P:  y_i = [x_i * (Qj/q_i)^-1]_{q_i} (centred),
// out_t = sum_i y_i [Qj/q_i]_t.
// The digit's own limbs are copied from the NTT-form input when `ntt` is set;
// otherwise they are not written and the key inner product reads them from
// the input (KipArgs::own).
// Table per digit j (stride tstride d2 entries): hinv[alpha], hat[le][alpha].
struct ModUpArgs {
  const u64* coef;        // c1 coefficient form of ct b: coef + b*coef_cs + l*N
  long long coef_cs;
  const u64* ntt;         // c1 NTT form of ct b: ntt + b*ntt_cs + l*N (null: own limbs not copied)
  long long ntt_cs;
  u64* ext;               // [B][beta][le][N]
  int b0;                 // first ct of the launch
  int beta, alpha, nl, le, logn;
  const d2* epq;          // [le] (q, 1/q) of the prime of extended limb l
  const d2* tab;          // per digit: alpha entries, then le rows of alpha (zero past the digit's limbs)
  int tstride;
};

template <int A, class X>
FENC_HD void modup_fbc_a(X& x, const ModUpArgs& a) {
  x.phase([&](int t) {
    const long long c = (long long)x.bx * x.nt + t;
    const int b = a.b0 + x.by / a.beta, j = x.by % a.beta;
    const int lo = j * a.alpha, hi = (lo + a.alpha < a.nl) ? lo + a.alpha : a.nl, ds = hi - lo;
    const d2* tab = a.tab + (long long)j * a.tstride;
    const long long N = 1LL << a.logn;
    u64* out = a.ext + ((long long)b * a.beta + j) * a.le * N;
    double y[A];
#pragma unroll
    for (int i = 0; i < A; i++) {
      y[i] = 0;
      if (i < ds) {
        const double q = a.epq[lo + i].x;
        const double v = u2d(a.coef[b * a.coef_cs + (lo + i) * N + c]);
        y[i] = centre(mulmod_c(v, tab[i].x, tab[i].y, q), q);   // v in [0, q): |v*w/q| < q
      }
    }
    if (a.ntt) {   // the digit's own limbs, copied from the NTT form
      u64 own[A];
#pragma unroll
      for (int i = 0; i < A; i++)
        if (i < ds) own[i] = a.ntt[b * a.ntt_cs + (lo + i) * N + c];
#pragma unroll
      for (int i = 0; i < A; i++)
        if (i < ds) out[(lo + i) * N + c] = own[i];
    }
    // the other limbs: no loads in this loop, so its stores need no wait
    for (int l = 0; l < a.le; l++) {
      if (l >= lo && l < hi) continue;
      const d2 pl = a.epq[l];
      const double q = pl.x, qi = pl.y;
      const d2* h = tab + a.alpha + (long long)l * a.alpha;
      double acc = 0;
      // A == alpha up to 8: every h[i] lies in the row and is zero, like
      // y[i], past the digit's limbs, so the products need no guard
#pragma unroll
      for (int i = 0; i < A; i++) {
        // |y| <= q_src/2 < 2^49: quotient below 2^49, product within 0.63q
        if (A <= 8 || i < ds) acc += mulmod_c(y[i], h[i].x, h[i].y, q);
        if ((i & 3) == 3) acc = red(acc, q, qi);
      }
      out[l * N + c] = d2u(norm(red(acc, q, qi), q));
    }
  });
}

template <class X>
FENC_HD void modup_fbc(X& x, const ModUpArgs& a) {
  with_count(a.alpha, [&](auto A) { modup_fbc_a<decltype(A)::value>(x, a); });
}

// ------------------------------------------------------------------ key inner product
// A group holds up to kKipOut outputs and the keys they use.  For every key
// the thread loads key_j once and applies it to each output that has an item
// for that key:  acc_o += sum_j sigma_g(ext_{ct,j}) * key_j.  One key shared
// by several outputs is the hoisted rotation of several ciphertexts by the
// same shift; several keys per output is the lazy-ModDown sum.
constexpr int kKipOut = 8;

struct KipKey {
  unsigned g;        // Galois element (1: identity)
  const u64* key;    // [ndig][2][nprimes][N]
  int item0;         // items[item0 + o], o < kKipOut: ext ct of output o of the group, or -1
};
struct KipGroup {
  int out0, nout;    // outputs out0 .. out0+nout-1
  int key0, nkey;    // keys key0 .. key0+nkey-1
};

struct KipArgs {
  const u64* ext;         // [B][beta][le][N]
  u64* acc;               // [nout][2][le][N]
  const KipGroup* groups;
  const KipKey* keys;
  const int* items;
  int g0;                 // first group of the launch
  int beta, le, logn, nprimes;
  const unsigned char* eprime;
  const d2* pq;
  // optional: acc_0 += P sigma_g(c0 of ct c0ct[item]) on the nl Q limbs, so
  // that ModDown of acc is the whole rotated ciphertext
  const int* c0ct;        // parallel to items, -1: none
  const u64* c0;          // c0 of input ct t at c0 + t * c0_cs
  long long c0_cs;
  const d2* pmod;         // [nl] P mod q_i
  int nl;
  int width;              // outputs per group slot row: 1, 2, 4 or kKipOut (>= every group's nout)
  // with own set, digit j's own limbs l in [j alpha, min((j+1) alpha, nl))
  // of an item are the input's NTT-form c1 limbs: own + own_ct[item] *
  // own_cs + l*N, with own_ct parallel to items (null: the item's ext ct),
  // and ModUp did not copy them into ext; with own null they are in ext
  const u64* own;
  long long own_cs;
  const int* own_ct;
  int alpha;
};

// A thread handles the coefficient pair (c, c+1), c even, with 16-byte
// accesses: sigma_g maps the evaluation points of a pair, w and -w, to w^g and
// -w^g, which are again a pair (m, m+1) in the bit-reversed order, swapped
// when auto_src(c) is odd.  W (1, 2, 4 or 8) is the launch's largest group
// padded to a power of two; padded slots read ct 0's words, which exist, and
// are computed but never stored, so every load is used and the loads in
// flight are counted exactly.
// OWN: the digits' own limbs come from the input (a.own), else all from ext;
// two kernels, so the plain one keeps its own register allocation.
template <int W, bool OWN, class X>
FENC_HD FENC_AI void kip_w(X& x, const KipArgs& a) {
  x.phase([&](int t) __attribute__((always_inline)) {
    const long long N = 1LL << a.logn;
    const long long c = 2 * ((long long)x.bx * x.nt + t);
    const int l = x.by;
    const KipGroup G = a.groups[a.g0 + x.bz];
    const int p = a.eprime[l];
    const double q = a.pq[p].x, qi = a.pq[p].y;
    const long long es = (long long)a.beta * a.le * N;   // ext ct stride
    double a0[W][2], a1[W][2];
#pragma unroll
    for (int o = 0; o < W; o++) a0[o][0] = a0[o][1] = a1[o][0] = a1[o][1] = 0;
    for (int kk = 0; kk < G.nkey; kk++) {
      const KipKey K = a.keys[G.key0 + kk];
      const long long src = (K.g == 1) ? c : (long long)auto_src((unsigned)c, K.g, a.logn);
      const long long m = src & ~1LL;
      const bool sw = (src & 1) != 0;
      // item lists are padded to kKipOut entries; -1 marks no item
      int ct[W], oc[W];
#pragma unroll
      for (int o = 0; o < W; o++) {
        ct[o] = a.items[K.item0 + o];
        ct[o] = ct[o] >= 0 ? ct[o] : 0;
        if constexpr (OWN) oc[o] = a.own_ct ? a.own_ct[K.item0 + o] : ct[o];   // loaded beside the item
      }
      for (int j = 0; j < a.beta; j++) {
        const u64* kj = K.key + ((long long)j * 2 * a.nprimes + p) * N + c;
        // every output's words for this digit are requested before any is used
        w2 v[W];
        if (OWN && l < a.nl && l >= j * a.alpha && l < (j + 1) * a.alpha) {   // own limb: the input's
          const u64* oj = a.own + (long long)l * N + m;
#pragma unroll
          for (int o = 0; o < W; o++) v[o] = ldg2(oj + (long long)oc[o] * a.own_cs);
        } else {
          const u64* ej = a.ext + ((long long)j * a.le + l) * N + m;
#pragma unroll
          for (int o = 0; o < W; o++) v[o] = ldg2(ej + (long long)ct[o] * es);
        }
        const w2 k0 = ldg2(kj), k1 = ldg2(kj + (long long)a.nprimes * N);
        const double k00 = u2d(k0[0]), k01 = u2d(k0[1]), k10 = u2d(k1[0]), k11 = u2d(k1[1]);
#pragma unroll
        for (int o = 0; o < W; o++) {
          const double e0 = u2d(sw ? v[o][1] : v[o][0]), e1 = u2d(sw ? v[o][0] : v[o][1]);
          // digit and key words in [0, q): |e*k/q| < q, sums within 1.5q
          a0[o][0] = red(a0[o][0] + mulmod(e0, k00, q, qi), q, qi);
          a0[o][1] = red(a0[o][1] + mulmod(e1, k01, q, qi), q, qi);
          a1[o][0] = red(a1[o][0] + mulmod(e0, k10, q, qi), q, qi);
          a1[o][1] = red(a1[o][1] + mulmod(e1, k11, q, qi), q, qi);
        }
      }
      if (a.c0 && l < a.nl) {
        int t0[W];
        bool use[W];
        w2 cv[W];
#pragma unroll
        for (int o = 0; o < W; o++) {
          t0[o] = a.c0ct[K.item0 + o];
          use[o] = t0[o] >= 0;
          t0[o] = use[o] ? t0[o] : 0;
        }
#pragma unroll
        for (int o = 0; o < W; o++) cv[o] = ldg2(a.c0 + (long long)t0[o] * a.c0_cs + (long long)l * N + m);
        // items without a folded c0 take the factor 0 (their words are still used)
#pragma unroll
        for (int o = 0; o < W; o++) {
          const double pw = use[o] ? a.pmod[l].x : 0.0, pwq = use[o] ? a.pmod[l].y : 0.0;
          const double e0 = u2d(sw ? cv[o][1] : cv[o][0]), e1 = u2d(sw ? cv[o][0] : cv[o][1]);
          a0[o][0] = red(a0[o][0] + mulmod_c(e0, pw, pwq, q), q, qi);
          a0[o][1] = red(a0[o][1] + mulmod_c(e1, pw, pwq, q), q, qi);
        }
      }
    }
#pragma unroll
    for (int o = 0; o < W; o++) {
      if (o >= G.nout) continue;
      u64* out = a.acc + (long long)(G.out0 + o) * 2 * a.le * N + (long long)l * N + c;
      stg2(out, d2u(norm(a0[o][0], q)), d2u(norm(a0[o][1], q)));
      stg2(out + (long long)a.le * N, d2u(norm(a1[o][0], q)), d2u(norm(a1[o][1], q)));
    }
  });
}

template <bool OWN, class X>
FENC_HD void kip_any(X& x, const KipArgs& a) {
  switch (a.width) {
    case 1: kip_w<1, OWN>(x, a); break;
    case 2: kip_w<2, OWN>(x, a); break;
    case 4: kip_w<4, OWN>(x, a); break;
    default: kip_w<kKipOut, OWN>(x, a); break;
  }
}
template <class X> FENC_HD void kip(X& x, const KipArgs& a) { kip_any<false>(x, a); }
template <class X> FENC_HD void kip_own(X& x, const KipArgs& a) { kip_any<true>(x, a); }

// ------------------------------------------------------------------ ModDown
// conv_i = sum_k [acc_{p_k} (P/p_k)^-1]_{p_k} [P/p_k]_{q_i}  (coefficient form,
// the bracket centred)
// Table: hinv[K], hat[nl][K].
struct ModDownArgs {
  const u64* acc;        // [nout][2][le][N], P limbs in coefficient form
  u64* conv;             // [nout][2][nl][N]
  int o0;                // first output of the launch
  int nl, le, K, logn;
  const d2* epq;         // [le] (q, 1/q) of the prime of extended limb l
  const d2* tab;
};

template <int KP, class X>
FENC_HD void moddown_fbc_k(X& x, const ModDownArgs& a) {
  x.phase([&](int t) {
    const long long N = 1LL << a.logn;
    const long long c = (long long)x.bx * x.nt + t;
    const long long op = 2LL * a.o0 + x.by;   // output * 2 + poly
    const u64* in = a.acc + op * a.le * N + c;
    double y[KP];
#pragma unroll
    for (int k = 0; k < KP; k++) {
      y[k] = 0;
      if (KP <= 8 || k < a.K) {
        const double q = a.epq[a.nl + k].x;
        // word in [0, q): |a*w/q| < q
        y[k] = centre(mulmod_c(u2d(in[(long long)(a.nl + k) * N]), a.tab[k].x, a.tab[k].y, q), q);
      }
    }
    u64* out = a.conv + op * a.nl * N + c;
    for (int i = 0; i < a.nl; i++) {
      const d2 pl = a.epq[i];
      const double q = pl.x, qi = pl.y;
      const d2* h = a.tab + a.K + (long long)i * a.K;
      double s = 0;
#pragma unroll
      for (int k = 0; k < KP; k++) {   // KP == K up to 8
        if (KP <= 8 || k < a.K) s += mulmod_c(y[k], h[k].x, h[k].y, q);   // |y| <= p/2 < 2^49
        if ((k & 3) == 3) s = red(s, q, qi);
      }
      out[(long long)i * N] = d2u(norm(red(s, q, qi), q));
    }
  });
}

template <class X>
FENC_HD void moddown_fbc(X& x, const ModDownArgs& a) {
  with_count(a.K, [&](auto KP) { moddown_fbc_k<decltype(KP)::value>(x, a); });
}

// out = (acc - conv) * P^-1 + base + sum_terms sigma_g(c0 of term ct)   (terms: poly 0 only)
// All cts are addressed as base pointer + index * ct stride; poly p of a ct
// starts at p * poly stride.
struct TailItem {
  int out;           // output ct index
  int base;          // base ct index or -1
  int add_off, add_n;
};
struct AddTerm {
  int ct;            // ct index in the add source
  unsigned g;
};
struct TailArgs {
  const u64* acc;    // [nout][2][le][N] (Q limbs NTT form)
  const u64* conv;   // [nout][2][nl][N] converted values (input of the NTT that applies the tail)
  const TailItem* items;
  const AddTerm* terms;
  int o0;
  int nl, le, logn;
  u64* out;  long long out_cs, out_ps;
  const u64* base;  long long base_cs, base_ps;
  const u64* add;   long long add_cs;
  const d2* pinv;    // [nl] (P^-1 mod q_i, /q)
  const d2* pq;
  const d2* bscale;  // [nl] factor of the base word (null: 1)
};

// Output word (o, poly, limb i, coefficient c) from the converted value cv
// (|cv| < q; |acc - cv| < 2q).  Two steps: the words of acc and base are
// loaded first (tail_load), the rest follows (tail_value).
// Both words are loaded unconditionally (without a base, word c of acc, which
// exists) and kept raw until tail_value, so the loads stay in flight together.
struct TailPre {
  u64 aw, bw;   // acc word; base word (unused without a base)
};
FENC_HD FENC_AI TailPre tail_load(const TailArgs& a, int o, int poly, int i, long long c) {
  const long long N = 1LL << a.logn;
  const TailItem I = a.items[o];
  const u64* ap = a.acc + ((long long)o * 2 + poly) * a.le * N + i * N + c;
  TailPre P;
  P.aw = ldg(ap);
  P.bw = ldg(I.base >= 0 ? a.base + I.base * a.base_cs + poly * a.base_ps + i * N + c : a.acc + c);
  return P;
}
FENC_HD FENC_AI void tail_value(const TailArgs& a, int o, int poly, int i, long long c, const TailPre& P, double cv,
                                double q, double qi) {
  const long long N = 1LL << a.logn;
  double r = mulmod_c(u2d(P.aw) - cv, a.pinv[i].x, a.pinv[i].y, q);   // |aw - cv| < 2q: quotient < 2^51
  const TailItem I = a.items[o];
  // with a factor: within 0.75q, so |r| < 1.75q before the added words
  if (I.base >= 0) r += a.bscale ? mulmod_c(u2d(P.bw), a.bscale[i].x, a.bscale[i].y, q) : u2d(P.bw);
  if (poly == 0)
    for (int k = 0; k < I.add_n; k++) {
      const AddTerm T = a.terms[I.add_off + k];
      const long long src = (T.g == 1) ? c : (long long)auto_src((unsigned)c, T.g, a.logn);
      r += u2d(a.add[T.ct * a.add_cs + i * N + src]);
      if ((k & 3) == 3) r = red(r, q, qi);
    }
  a.out[I.out * a.out_cs + poly * a.out_ps + i * N + c] = d2u(norm(red(r, q, qi), q));
}

// ModDown by P q_l (a relinearisation and the rescale after it in one base
// conversion): the q_l limb of the converted sum is acc_l + P base_l, so that
// limb of acc (NTT form, not read by the tail) takes the base's share before
// its inverse NTT with the special primes' limbs.  One thread per
// coefficient; rows: output * 2 + poly.
struct RsPrepArgs {
  u64* acc;                 // [nout][2][le][N]
  const u64* base;  long long base_cs, base_ps;
  const TailItem* items;
  int o0, nl, le, logn;
  d2 pmod, pq;              // (P mod q_l, /q_l), (q_l, 1/q_l)
};
template <class X>
FENC_HD void rs_prep(X& x, const RsPrepArgs& a) {
  x.phase([&](int t) {
    const long long N = 1LL << a.logn;
    const long long c = (long long)x.bx * x.nt + t;
    const int o = a.o0 + x.by / 2, poly = x.by & 1;
    const double q = a.pq.x, qi = a.pq.y;
    u64* ap = a.acc + ((long long)(o * 2 + poly) * a.le + (a.nl - 1)) * N + c;
    const u64* bp = a.base + a.items[o].base * a.base_cs + poly * a.base_ps + (long long)(a.nl - 1) * N + c;
    // acc word in [0, q), product within 0.75q
    const double v = u2d(ldg(ap)) + mulmod_c(u2d(ldg(bp)), a.pmod.x, a.pmod.y, q);
    *ap = d2u(norm(red(v, q, qi), q));
  });
}

// The tail is the epilogue of the forward row pass that finishes the NTT of
// the converted values (rows: [output][poly][limb], limb = prime index), so
// the converted values never return to memory.
FENC_HD FENC_AI TailPre epi_load(const TailArgs& a, int row, long long c, double, double) {
  const int i = row % a.nl, grp = row / a.nl;
  return tail_load(a, a.o0 + (grp >> 1), grp & 1, i, c);
}
FENC_HD FENC_AI void epi_finish(const TailArgs& a, int row, long long c, const TailPre& P, double v, double q,
                                double qi) {
  const int i = row % a.nl, grp = row / a.nl;
  tail_value(a, a.o0 + (grp >> 1), grp & 1, i, c, P, v, q, qi);
}

struct NttMdArgs {
  NttArgs n;
  TailArgs t;
};
template <int RB, class X>
FENC_HD void ntt_fwd_rows_md_rb(X& x, const NttMdArgs& a) {
  const int p = a.n.pm.p[x.by % a.n.pm.n];
  if (p == kSkip) return;
  with_pass(a.n.n2, [&](auto P) { ntt_rows_pass<false, decltype(P)::value, RB>(x, a.n, p, &a.t); });
}
template <class X> FENC_HD void ntt_fwd_rows_md(X& x, const NttMdArgs& a) { ntt_fwd_rows_md_rb<3>(x, a); }
template <class X> FENC_HD void ntt_fwd_rows16_md(X& x, const NttMdArgs& a) { ntt_fwd_rows_md_rb<4>(x, a); }

// ------------------------------------------------------------------ rescale
// last: coefficient form of limb l (rows [B][2]); lift centred value to each q_i, i < l
struct LiftArgs {
  const u64* last;   // [B*2][N]
  int nl, logn;      // nl: limbs the value is lifted to (rows per ct and poly of the NTT it feeds)
  double ql;
  const d2* pq;
};

// The lift as the prologue of the forward column pass over the lifted rows
// ([ct * 2 + poly][limb]): the rows of one ct and poly share the last limb's
// words, so the lifted values are never written.
FENC_HD inline double pro_load(const LiftArgs& a, int row, long long c, double q, double qi) {
  const long long N = 1LL << a.logn;
  double v = u2d(a.last[(long long)(row / a.nl) * N + c]);
  if (v > (a.ql - 1) * 0.5) v -= a.ql;   // centred representative
  return red(v, q, qi);
}

struct NttLiftArgs {
  NttArgs n;
  LiftArgs l;
};
template <int RB, class X>
FENC_HD void ntt_fwd_cols_lift_rb(X& x, const NttLiftArgs& a) {
  const int p = a.n.pm.p[x.by % a.n.pm.n];
  if (p == kSkip) return;
  with_pass(a.n.n1, [&](auto P) { ntt_cols_pass<false, decltype(P)::value, RB>(x, a.n, p, &a.l); });
}
template <class X> FENC_HD void ntt_fwd_cols_lift(X& x, const NttLiftArgs& a) { ntt_fwd_cols_lift_rb<3>(x, a); }
template <class X> FENC_HD void ntt_fwd_cols16_lift(X& x, const NttLiftArgs& a) { ntt_fwd_cols_lift_rb<4>(x, a); }

struct RescaleTailArgs {
  const u64* in;     // [B][2][nl+1][N]
  const u64* lift;   // [B*2][nl][N] lifted last limb (input of the NTT that applies the tail)
  u64* out;          // [B][2][nl][N]
  int nl, logn;
  const d2* qlinv;   // [nl]
  const d2* pq;
};

// The rescale tail as the epilogue of the forward row pass that finishes the
// NTT of the lifted last limb (rows: [ct * 2 + poly][limb]); w in [-q/2, q/2].
FENC_HD FENC_AI u64 epi_load(const RescaleTailArgs& a, int row, long long c, double, double) {
  const long long N = 1LL << a.logn;
  const int i = row % a.nl, r = row / a.nl;   // r = ct*2 + poly
  return ldg(a.in + ((long long)r * (a.nl + 1) + i) * N + c);
}
FENC_HD FENC_AI void epi_finish(const RescaleTailArgs& a, int row, long long c, u64 vw, double w, double q, double) {
  const long long N = 1LL << a.logn;
  const int i = row % a.nl, r = row / a.nl;
  // vw - w in (-q/2 - 1, 1.5q + 1): quotient within (-q/2, 1.5q), product < q
  a.out[((long long)r * a.nl + i) * N + c] = d2u(norm(mulmod_c(u2d(vw) - w, a.qlinv[i].x, a.qlinv[i].y, q), q));
}

struct NttRsArgs {
  NttArgs n;
  RescaleTailArgs t;
};
template <int RB, class X>
FENC_HD void ntt_fwd_rows_rs_rb(X& x, const NttRsArgs& a) {
  const int p = a.n.pm.p[x.by % a.n.pm.n];
  if (p == kSkip) return;
  with_pass(a.n.n2, [&](auto P) { ntt_rows_pass<false, decltype(P)::value, RB>(x, a.n, p, &a.t); });
}
template <class X> FENC_HD void ntt_fwd_rows_rs(X& x, const NttRsArgs& a) { ntt_fwd_rows_rs_rb<3>(x, a); }
template <class X> FENC_HD void ntt_fwd_rows16_rs(X& x, const NttRsArgs& a) { ntt_fwd_rows_rs_rb<4>(x, a); }

// ------------------------------------------------------------------ lift to the extended basis
// out[t] = P x_t on the nl Q limbs and 0 on the K special limbs ([2][le][N],
// NTT form): ModDown of it gives x_t back, so unrotated inputs join linear
// combinations taken in Q_l U P.
struct LiftPqArgs {
  const u64* in;  long long in_cs;   // [n][2][nl][N]
  u64* out;  long long out_cs;       // [n][2][le][N]
  int nl, le, logn;
  const d2* pmod;                    // [nl] P mod q_i
  const d2* pq;
};

template <class X>
FENC_HD void lift_pq(X& x, const LiftPqArgs& a) {
  x.phase([&](int t) {
    const long long N = 1LL << a.logn;
    const long long c = (long long)x.bx * x.nt + t;
    const int l = x.by % a.le, poly = x.by / a.le, b = x.bz;
    u64* o = a.out + b * a.out_cs + ((long long)poly * a.le + l) * N + c;
    if (l >= a.nl) {
      *o = 0;
      return;
    }
    const double q = a.pq[l].x;
    const double v = u2d(a.in[b * a.in_cs + ((long long)poly * a.nl + l) * N + c]);
    *o = d2u(norm(mulmod_c(v, a.pmod[l].x, a.pmod[l].y, q), q));
  });
}

// ------------------------------------------------------------------ linear combinations
// A class is a set of up to kMacOut outputs with the same input terms, each
// output with its own integer weights and its own plaintext per group (a small
// modular GEMM followed by a plaintext product):
//   out_o = sum_g pt_{g,o} (.) ( sum_{t in g} w_{t,o} * in_t )   (NTT form, both polys)
// Each input word is loaded once for all outputs of the class.  Input index
// t < na addresses in_a + t*a_cs, otherwise in_b + (t-na)*b_cs.  A null
// plaintext means no product.
constexpr int kMacOut = 8;
// the kernels' width dispatch (1, 2, 4, default) takes the default for 8
static_assert(kMacOut == 8, "class rows are 1, 2, 4 or 8 wide");

struct MacClass {
  int g0, ng;        // groups g0 .. g0+ng-1 (terms shared by the outputs)
  int o0, nout;      // cls_out[o0 .. o0+nout-1]: output ct indices
  int w0;            // weights: ew[limb][w0 + term_rank * width + o]
  int m0;            // plaintexts: mask[m0 + group_rank * width + o]
};

struct GmacArgs {
  const u64* in_a; long long a_cs, a_ps; int na;
  const u64* in_b; long long b_cs, b_ps;
  int nl_a;                  // limbs of the A inputs: A terms read nothing at limbs >= nl_a
  u64* out; long long out_cs, out_ps;
  int c0;                    // first class of the launch
  int width;                 // 1, 2, 4, 8 or 16: outputs per class row (nout <= width; rows zero-padded)
  const MacClass* cls;
  const int* cls_out;
  const u64* const* mask;    // per (class, group, output) plaintext [nl][N] or null
  const int* toff;           // [ngroups+1] term ranges
  const int* tin;            // [nterms] input index
  const d2* ew;              // [nl][ews] weight residues (w mod q, fl(w/q))
  long long ews;
  const double* wc;          // [ews] signed weight codes of the small-code classes (any limb)
  int chunk;                 // terms per chunk: kMacChunk or 4
  int nl, logn;
  const unsigned char* eprime;   // prime index of limb i (null: i)
  const d2* pq;
};

// Grid (N/256, nl, 2 * classes): z = class * 2 + poly, launched in the
// XCD-aware order so both polys and neighbouring classes of one tile share an
// L2 (plaintexts and shared inputs are fetched once).
// Classes whose weight codes are all below 2^23 in magnitude (split-scale
// weights) take exact products without a modular reduction per term: the
// input word is split into 25-bit halves, hi * w and lo * w are exact binary64
// integers below 2^48, and 16 of them are summed before one reduction.  The
// weight table then holds the signed code itself (y unused).
constexpr int kFastWBits = 23;

constexpr int kMacChunk = 8;   // input words requested together (classes with small groups: 4)

// Plaintext products of a class: none, one plaintext per group shared by every
// output of the class, or one per (group, output).
enum { kPtNone = 0, kPtShared = 1, kPtEach = 2 };

// Requests the input words of terms k .. k+cnt-1 (cnt <= CH <= kMacChunk).  The term
// table carries kMacChunk spare entries, so a whole chunk of indices is read
// at once; every slot of the chunk issues one load (slots past cnt read the
// word of input ts, which exists), so the loads in flight are counted exactly.
// A inputs have no words at limbs >= nl_a: off_a then addresses limb 0, and
// the weights of A terms are zero at those limbs.
template <int CH>
FENC_HD FENC_AI void mac_fetch(const GmacArgs& a, int k, int cnt, int ts, long long off_a, long long off_b,
                               u64 (&v)[CH]) {
  int ti[CH];
#pragma unroll
  for (int j = 0; j < CH; j++) ti[j] = a.tin[k + j];
#pragma unroll
  for (int j = 0; j < CH; j++) {
    const int tj = j < cnt ? ti[j] : ts;
    const u64* p = tj < a.na ? a.in_a + tj * a.a_cs + off_a : a.in_b + (tj - a.na) * a.b_cs + off_b;
    v[j] = ldg(p);
  }
}

// Requests the plaintext word(s) of one group (mg: its W plaintext pointers);
// for a null plaintext the word at `safe` is read and never used.
template <int W, int PTM>
FENC_HD FENC_AI void mac_fetch_pt(const u64* const* mg, bool use, long long off, const u64* safe,
                                  u64 (&m)[PTM == kPtEach ? W : 1]) {
  constexpr int NM = PTM == kPtEach ? W : 1;
#pragma unroll
  for (int o = 0; o < NM; o++) {
    const u64* p = use ? mg[o] : nullptr;
    m[o] = ldg(p ? p + off : safe);
  }
}

// Adds the cnt terms of one chunk (weights w[j * W + o]) into the group sums.
// FAST: acc/acc2 hold the sums of hi*w and lo*w, reduced once more than
// 16 - CH terms are in them (at most 16 unreduced products of < 2^48);
// otherwise acc holds a sum of modular products reduced every 5 terms.
template <int W, bool FAST, int CH>
FENC_HD FENC_AI void mac_terms(const u64 (&v)[CH], int cnt, const d2* w, const double* wc, double q,
                               double qi, int& n, double (&acc)[W], double (&acc2)[W]) {
#pragma unroll
  for (int j = 0; j < CH; j++) {
    if (j >= cnt) break;
    if constexpr (FAST) {
      const double* cj = wc + j * W;
      const double vh = u2d(v[j] >> 25), vl = u2d(v[j] & 0x1FFFFFFull);
#pragma unroll
      for (int o = 0; o < W; o++) {
        acc[o] = fma(vh, cj[o], acc[o]);
        acc2[o] = fma(vl, cj[o], acc2[o]);
      }
    } else {
      const d2* wj = w + j * W;
      const double vv = u2d(v[j]);
#pragma unroll
      for (int o = 0; o < W; o++) acc[o] += mulmod_c(vv, wj[o].x, wj[o].y, q);   // vv in [0, q)
      if (++n == 5) {
#pragma unroll
        for (int o = 0; o < W; o++) acc[o] = red(acc[o], q, qi);
        n = 0;
      }
    }
  }
  if constexpr (FAST) {
    n += cnt;
    if (n > 16 - CH) {
#pragma unroll
      for (int o = 0; o < W; o++) {
        acc[o] = red(acc[o], q, qi);
        acc2[o] = red(acc2[o], q, qi);
      }
      n = 0;
    }
  }
}

// End of a group: fold its sums into r, through its plaintext word(s) m.
template <int W, int PTM, bool FAST>
FENC_HD FENC_AI void mac_end_group(const u64* const* mg, double q, double qi, const u64 (&m)[PTM == kPtEach ? W : 1],
                                   double (&acc)[W], double (&acc2)[W], double (&r)[W]) {
  const double t25 = 33554432.0, t25q = t25 * qi;   // 2^25 < q
  double ms = 0;
  if constexpr (PTM == kPtShared) ms = u2d(m[0]);
#pragma unroll
  for (int o = 0; o < W; o++) {
    double sv;
    // reduced sums within q/2 + 1 times 2^25 or a word in [0, q): quotients below 2^50
    if constexpr (FAST) sv = red(mulmod_c(red(acc[o], q, qi), t25, t25q, q) + red(acc2[o], q, qi), q, qi);
    else sv = red(acc[o], q, qi);
    if constexpr (PTM == kPtShared) {
      if (mg[0]) sv = mulmod(sv, ms, q, qi);
    } else if constexpr (PTM == kPtEach) {
      if (mg[o]) sv = mulmod(sv, u2d(m[o]), q, qi);
    }
    r[o] = red(r[o] + sv, q, qi);
    acc[o] = 0;
    acc2[o] = 0;
  }
}

// Common set-up of a MAC thread: its coefficient, limb, poly and class.
struct MacThread {
  long long N, c, off_a, off_b, off_pt;
  int i, poly, k0, gend, nterm;
  int ts;              // first term's input: the spare loads read its word
  const u64* safe;     // address of that word
  bool a_here;
  double q, qi;
  MacClass K;
};

template <class X>
FENC_HD FENC_AI MacThread mac_thread(X& x, int t, const GmacArgs& a) {
  MacThread m;
  m.N = 1LL << a.logn;
  m.c = (long long)x.bx * x.nt + t;
  m.i = x.by;
  m.poly = x.bz & 1;
  m.K = a.cls[a.c0 + (x.bz >> 1)];
  const int pi = a.eprime ? a.eprime[m.i] : m.i;
  m.q = a.pq[pi].x;
  m.qi = a.pq[pi].y;
  m.a_here = m.i < a.nl_a;
  m.off_a = m.poly * a.a_ps + (m.a_here ? m.i * m.N : 0) + m.c;
  m.off_b = m.poly * a.b_ps + m.i * m.N + m.c;
  m.off_pt = m.i * m.N + m.c;
  m.gend = m.K.g0 + m.K.ng;
  m.k0 = m.K.ng > 0 ? a.toff[m.K.g0] : 0;
  m.nterm = m.K.ng > 0 ? a.toff[m.gend] - m.k0 : 0;
  m.ts = a.tin[m.k0];
  m.safe = m.ts < a.na ? a.in_a + m.ts * a.a_cs + m.off_a : a.in_b + (m.ts - a.na) * a.b_cs + m.off_b;
  return m;
}

template <int W, class X>
FENC_HD FENC_AI void mac_store(const GmacArgs& a, const MacThread& m, const double (&r)[W]) {
#pragma unroll
  for (int o = 0; o < W; o++) {
    if (o >= m.K.nout) continue;
    a.out[a.cls_out[m.K.o0 + o] * a.out_cs + m.poly * a.out_ps + m.i * m.N + m.c] = d2u(norm(r[o], m.q));
  }
}

// One MAC kernel body for the general forms: W outputs per class row, PTM
// plaintext products, FAST small signed codes (see kFastWBits).  The terms of
// each group are walked in chunks of up to CH, in two alternating
// buffers: the words of the next chunk (with its group's plaintext words when
// it ends its group) are requested before the current chunk is used.
template <int W, int PTM, int CH>
struct MacBuf {
  u64 v[CH];
  u64 m[PTM == kPtEach ? W : 1];
};

// Walk state of one MAC thread: the chunk (g, k) of group g ending at ge, the
// unreduced term count n and the sums.
template <int W>
struct MacState {
  MacThread T;
  const d2* ew;
  const double* wc;
  const u64* const* mk;
  int g, k, ge, n;
  bool done;
  double r[W], acc[W], acc2[W];
};

// Requests chunk (g, k) of group g ending at ge (with the group's plaintext
// words when the chunk ends the group).
template <int W, int PTM, int CH>
FENC_HD FENC_AI void mac_chunk_fetch(const GmacArgs& a, const MacState<W>& S, MacBuf<W, PTM, CH>& b, int g, int k,
                                     int ge) {
  const int cnt = ge - k < CH ? ge - k : CH;
  mac_fetch(a, k, cnt, S.T.ts, S.T.off_a, S.T.off_b, b.v);
  if constexpr (PTM != kPtNone)
    mac_fetch_pt<W, PTM>(S.mk + (long long)(g - S.T.K.g0) * W, k + cnt >= ge, S.T.off_pt, S.T.safe, b.m);
}

// Requests the next chunk into nxt (past the class end, the first chunk again,
// never used), then adds the current chunk cur and closes its group if it ends.
template <int W, int PTM, bool FAST, int CH>
FENC_HD FENC_AI void mac_step(const GmacArgs& a, MacState<W>& S, const MacBuf<W, PTM, CH>& cur,
                              MacBuf<W, PTM, CH>& nxt) {
  const int cnt = S.ge - S.k < CH ? S.ge - S.k : CH;
  const bool last = S.k + cnt >= S.ge;
  int kn = S.k + cnt, gn = S.g, gen = S.ge;
  if (last) {
    gn = S.g + 1;
    if (gn < S.T.gend) gen = a.toff[gn + 1];
  }
  const bool more = gn < S.T.gend;
  if (more) mac_chunk_fetch(a, S, nxt, gn, kn, gen);
  else mac_chunk_fetch(a, S, nxt, S.T.K.g0, S.T.k0, S.T.k0);
  const long long w = (long long)(S.k - S.T.k0) * W;
  mac_terms<W, FAST, CH>(cur.v, cnt, S.ew + w, S.wc + w, S.T.q, S.T.qi, S.n, S.acc, S.acc2);
  if (last) {
    mac_end_group<W, PTM, FAST>(S.mk + (long long)(S.g - S.T.K.g0) * W, S.T.q, S.T.qi, cur.m, S.acc, S.acc2, S.r);
    S.n = 0;
  }
  S.k = kn;
  S.g = gn;
  S.ge = gen;
  S.done = !more;
}

template <int W, int PTM, bool FAST, int CH, class X>
FENC_HD FENC_AI void gmac_body(X& x, const GmacArgs& a) {
  x.phase([&](int t) __attribute__((always_inline)) {
    MacState<W> S;
    S.T = mac_thread(x, t, a);
    S.ew = a.ew + (long long)S.T.i * a.ews + S.T.K.w0;
    S.wc = a.wc + S.T.K.w0;
    S.mk = a.mask + S.T.K.m0;
#pragma unroll
    for (int o = 0; o < W; o++) S.r[o] = S.acc[o] = S.acc2[o] = 0;
    if (S.T.nterm > 0) {
      S.g = S.T.K.g0;
      S.k = S.T.k0;
      S.ge = a.toff[S.g + 1];
      S.n = 0;
      S.done = false;
      MacBuf<W, PTM, CH> A, B;
      mac_chunk_fetch(a, S, A, S.g, S.k, S.ge);
      for (;;) {
        mac_step<W, PTM, FAST, CH>(a, S, A, B);
        if (S.done) break;
        mac_step<W, PTM, FAST, CH>(a, S, B, A);
        if (S.done) break;
      }
    }
    mac_store<W, X>(a, S.T, S.r);
  });
}

// Diagonal form: every group is one term of weight 1 with its own plaintext
// per output (materialised diagonals, FC diagonals, compress masks):
//   out_o = sum_g pt_{g,o} (.) in_g
// Groups alternate between two buffers: the next group's input and plaintext
// words are requested before the current group's products.  The sums are
// reduced every 4 groups (|r| < q/2 + 4q).
template <int W>
struct DiagBuf {
  u64 v[1];
  u64 m[W];
};

template <int W>
FENC_HD FENC_AI void diag_fetch(const GmacArgs& a, const MacThread& T, const u64* const* mk, int g, DiagBuf<W>& b) {
  mac_fetch(a, a.toff[g], 1, T.ts, T.off_a, T.off_b, b.v);
  mac_fetch_pt<W, kPtEach>(mk + (long long)(g - T.K.g0) * W, true, T.off_pt, T.safe, b.m);
}

// Adds group g from cur after requesting group g + 1 (past the class end, the
// first group again, never used) into nxt.
template <int W>
FENC_HD FENC_AI bool diag_step(const GmacArgs& a, const MacThread& T, const u64* const* mk, int& g, int& n,
                               const DiagBuf<W>& cur, DiagBuf<W>& nxt, double (&r)[W]) {
  const bool more = g + 1 < T.gend;
  diag_fetch(a, T, mk, more ? g + 1 : T.K.g0, nxt);
  const double vv = u2d(cur.v[0]);
#pragma unroll
  for (int o = 0; o < W; o++) r[o] += mulmod(vv, u2d(cur.m[o]), T.q, T.qi);   // both words in [0, q)
  if (++n == 4) {
#pragma unroll
    for (int o = 0; o < W; o++) r[o] = red(r[o], T.q, T.qi);
    n = 0;
  }
  g++;
  return more;
}

template <int W, class X>
FENC_HD FENC_AI void gmac_diag_body(X& x, const GmacArgs& a) {
  x.phase([&](int t) __attribute__((always_inline)) {
    const MacThread T = mac_thread(x, t, a);
    const u64* const* mk = a.mask + T.K.m0;
    double r[W];
#pragma unroll
    for (int o = 0; o < W; o++) r[o] = 0;
    if (T.nterm > 0) {
      DiagBuf<W> A, B;
      int g = T.K.g0, n = 0;
      diag_fetch(a, T, mk, g, A);
      for (;;) {
        if (!diag_step(a, T, mk, g, n, A, B, r)) break;
        if (!diag_step(a, T, mk, g, n, B, A, r)) break;
      }
#pragma unroll
      for (int o = 0; o < W; o++) r[o] = red(r[o], T.q, T.qi);
    }
    mac_store<W, X>(a, T, r);
  });
}

// Single-term form: every group is one weighted term with the class's shared
// plaintext (or none), as in depthwise convolutions where each position mask
// multiplies one rotated copy:
//   out_o = sum_g pt_g (.) (w_{g,o} * in_g)
// Each term is two modular products (weight, then plaintext word) instead of
// the split-and-accumulate of the general form, whose exact sums pay off only
// when a group holds many terms.  Groups alternate between two buffers (the
// next group's words are requested first); sums are reduced every 4 groups.
struct OneBuf {
  u64 v[1];
  u64 m[1];
};

FENC_HD FENC_AI void one_fetch(const GmacArgs& a, const MacThread& T, const u64* const* mk, int W, int g,
                               OneBuf& b) {
  mac_fetch(a, a.toff[g], 1, T.ts, T.off_a, T.off_b, b.v);
  const u64* p = mk[(long long)(g - T.K.g0) * W];
  b.m[0] = ldg(p ? p + T.off_pt : T.safe);
}

template <int W>
FENC_HD FENC_AI bool one_step(const GmacArgs& a, const MacThread& T, const d2* ew, const u64* const* mk, int& g,
                              int& n, const OneBuf& cur, OneBuf& nxt, double (&r)[W]) {
  const bool more = g + 1 < T.gend;
  one_fetch(a, T, mk, W, more ? g + 1 : T.K.g0, nxt);
  const double vv = u2d(cur.v[0]), ms = u2d(cur.m[0]);
  const bool has_pt = mk[(long long)(g - T.K.g0) * W] != nullptr;
  const d2* w = ew + (long long)(g - T.K.g0) * W;   // one term per group: term rank = group rank
#pragma unroll
  for (int o = 0; o < W; o++) {
    double t = mulmod_c(vv, w[o].x, w[o].y, T.q);    // vv in [0, q): |t| <= 0.75q
    if (has_pt) t = mulmod(t, ms, T.q, T.qi);        // |t * ms / q| < q
    r[o] += t;
  }
  if (++n == 4) {
#pragma unroll
    for (int o = 0; o < W; o++) r[o] = red(r[o], T.q, T.qi);
    n = 0;
  }
  g++;
  return more;
}

template <int W, class X>
FENC_HD FENC_AI void gmac_one_body(X& x, const GmacArgs& a) {
  x.phase([&](int t) __attribute__((always_inline)) {
    const MacThread T = mac_thread(x, t, a);
    const u64* const* mk = a.mask + T.K.m0;
    const d2* ew = a.ew + (long long)T.i * a.ews + T.K.w0;
    double r[W];
#pragma unroll
    for (int o = 0; o < W; o++) r[o] = 0;
    if (T.nterm > 0) {
      OneBuf A, B;
      int g = T.K.g0, n = 0;
      one_fetch(a, T, mk, W, g, A);
      for (;;) {
        if (!one_step<W>(a, T, ew, mk, g, n, A, B, r)) break;
        if (!one_step<W>(a, T, ew, mk, g, n, B, A, r)) break;
      }
#pragma unroll
      for (int o = 0; o < W; o++) r[o] = red(r[o], T.q, T.qi);
    }
    mac_store<W, X>(a, T, r);
  });
}

// Classes with one plaintext per (group, output) hold at most kMacOutEach
// outputs (their plaintext words take registers per output).
constexpr int kMacOutEach = 4;

template <int PTM, bool FAST, int CH, class X>
FENC_HD FENC_AI void gmac_width(X& x, const GmacArgs& a) {
  constexpr int WMAX = PTM == kPtEach ? kMacOutEach : kMacOut;
  switch (a.width) {
    case 1: gmac_body<1, PTM, FAST, CH>(x, a); break;
    case 2: gmac_body<2, PTM, FAST, CH>(x, a); break;
    case 4: gmac_body<4, PTM, FAST, CH>(x, a); break;
    default: gmac_body<WMAX, PTM, FAST, CH>(x, a); break;   // width 8 (kMacOut)
  }
}
template <int PTM, bool FAST, class X>
FENC_HD void gmac_any(X& x, const GmacArgs& a) {
  if (a.chunk == kMacChunk) gmac_width<PTM, FAST, kMacChunk>(x, a);
  else gmac_width<PTM, FAST, 4>(x, a);
}
// classes without plaintext products
template <class X>
FENC_HD void gmac(X& x, const GmacArgs& a) { gmac_any<kPtNone, false>(x, a); }
// one plaintext per group for the whole class
template <class X>
FENC_HD void gmac_pt(X& x, const GmacArgs& a) { gmac_any<kPtShared, false>(x, a); }
// one plaintext per (group, output)
template <class X>
FENC_HD void gmac_ptv(X& x, const GmacArgs& a) { gmac_any<kPtEach, false>(x, a); }
// the same three with small weight codes (|code| < 2^23)
template <class X>
FENC_HD void gmac_fast(X& x, const GmacArgs& a) { gmac_any<kPtNone, true>(x, a); }
template <class X>
FENC_HD void gmac_pt_fast(X& x, const GmacArgs& a) { gmac_any<kPtShared, true>(x, a); }
template <class X>
FENC_HD void gmac_ptv_fast(X& x, const GmacArgs& a) { gmac_any<kPtEach, true>(x, a); }
// single-term classes
template <class X>
FENC_HD void gmac_one(X& x, const GmacArgs& a) {
  switch (a.width) {
    case 1: gmac_one_body<1>(x, a); break;
    case 2: gmac_one_body<2>(x, a); break;
    case 4: gmac_one_body<4>(x, a); break;
    default: gmac_one_body<kMacOut>(x, a); break;   // width 8 (kMacOut)
  }
}
// diagonal classes
template <class X>
FENC_HD void gmac_diag(X& x, const GmacArgs& a) {
  switch (a.width) {
    case 1: gmac_diag_body<1>(x, a); break;
    case 2: gmac_diag_body<2>(x, a); break;
    case 4: gmac_diag_body<4>(x, a); break;
    default: gmac_diag_body<kMacOut>(x, a); break;   // width 8 (kMacOut)
  }
}

// ------------------------------------------------------------------ tensor / key / encryption
// Tensor product of ciphertexts a and b (b == a for a square), times the
// integer k: (d0, d1, d2) = k (a0 b0, a0 b1 + a1 b0, a1 b1); d0, d1 into out
// (ct [2][nl][N]), d2 into d2buf [nl][N].
// out = k (a0 b0, a0 b1 + a1 b0) [+ k1 x + k0], d2buf = k a1 b1.  The optional
// linear term of the activation (x with its own strides, possibly more limbs:
// limb drop; k0 on poly 0 only) is added here, so it needs no pass of its own.
// With kb1 set, b is not read but formed from x: b = kb1 x + kb0 (kb0 on poly
// 0), the cubic's second factor.
struct SquareArgs {
  const u64* in;
  const u64* in_b;
  u64* out;
  u64* d2buf;
  int nl, logn;
  long long ct_stride;   // elements per ct (inputs and out)
  const d2* k;           // [nl] (k mod q_i, /q)
  const d2* pq;
  const u64* lx;         // x (null: no linear term and no formed b)
  long long lx_cs, lx_ps;
  const d2* k1;          // [nl] null: no linear term
  const d2* k0;          // [nl]
  const d2* kb1;         // [nl] null: b read from in_b
  const d2* kb0;         // [nl]
};

template <class X>
FENC_HD void tensor_square(X& x, const SquareArgs& a) {
  x.phase([&](int t) {
    const long long N = 1LL << a.logn;
    const long long c = (long long)x.bx * x.nt + t;
    const int i = x.by, b = x.bz;
    const double q = a.pq[i].x, qi = a.pq[i].y;
    const u64* pa = a.in + b * a.ct_stride + i * N + c;
    const u64* pb = a.in_b + b * a.ct_stride + i * N + c;
    const double a0 = u2d(pa[0]), a1 = u2d(pa[a.nl * N]);
    double b0, b1;
    if (a.kb1) {   // b = kb1 x + kb0, each word in [0, q) like a stored one
      const u64* px = a.lx + b * a.lx_cs + i * N + c;
      b0 = norm(red(mulmod_c(u2d(px[0]), a.kb1[i].x, a.kb1[i].y, q) + a.kb0[i].x, q, qi), q);
      b1 = norm(red(mulmod_c(u2d(px[a.lx_ps]), a.kb1[i].x, a.kb1[i].y, q), q, qi), q);
    } else {
      b0 = u2d(pb[0]);
      b1 = u2d(pb[a.nl * N]);
    }
    u64* out = a.out + b * a.ct_stride + i * N + c;
    const d2 k = a.k[i];
    const double m01 = mulmod(a0, b1, q, qi) + mulmod(a1, b0, q, qi);   // words in [0, q)
    double o0 = mulmod_c(mulmod(a0, b0, q, qi), k.x, k.y, q), o1 = mulmod_c(m01, k.x, k.y, q);
    if (a.lx && a.k1) {   // each term within q: the sums stay within 3q, reduced once
      const u64* px = a.lx + b * a.lx_cs + i * N + c;
      const double x0 = px == pa ? a0 : u2d(px[0]), x1 = px == pa ? a1 : u2d(px[a.lx_ps]);
      o0 = red(o0 + mulmod_c(x0, a.k1[i].x, a.k1[i].y, q) + a.k0[i].x, q, qi);
      o1 = red(o1 + mulmod_c(x1, a.k1[i].x, a.k1[i].y, q), q, qi);
    }
    out[0] = d2u(norm(o0, q));
    out[a.nl * N] = d2u(norm(o1, q));
    a.d2buf[(long long)b * a.nl * N + i * N + c] = d2u(norm(mulmod_c(mulmod(a1, b1, q, qi), k.x, k.y, q), q));
  });
}

// out = base + k1 * x + k0 (k0 on poly 0 only: the constant polynomial k0 in
// NTT form); base may be null; x may have more limbs than out (limb drop).
struct LinArgs {
  const u64* x;  long long x_cs, x_ps;
  const u64* base;  long long b_cs, b_ps;
  u64* out;  long long o_cs, o_ps;
  int nl, logn;
  const d2* k1;          // [nl]
  const d2* k0;          // [nl]
  const d2* pq;
};

template <class X>
FENC_HD void lin_comb(X& x, const LinArgs& a) {
  x.phase([&](int t) {
    const long long N = 1LL << a.logn;
    const long long c = (long long)x.bx * x.nt + t;
    const int i = x.by % a.nl, poly = x.by / a.nl, b = x.bz;
    const double q = a.pq[i].x, qi = a.pq[i].y;
    const double xv = u2d(a.x[b * a.x_cs + poly * a.x_ps + i * N + c]);
    double r = mulmod_c(xv, a.k1[i].x, a.k1[i].y, q);
    if (a.base) r += u2d(a.base[b * a.b_cs + poly * a.b_ps + i * N + c]);
    if (poly == 0) r += a.k0[i].x;
    a.out[b * a.o_cs + poly * a.o_ps + i * N + c] = d2u(norm(red(r, q, qi), q));
  });
}

// b = -a*s + e + gadget * s'   (all NTT form over prime p); rows: digit*np + prime
struct KeyArgs {
  const u64* a;      // [ndig][np][N]
  const u64* e;      // [ndig][np][N]
  const u64* s;      // [np][N] secret, NTT form
  const u64* sp;     // [np][N] target secret s' (NTT form)
  u64* key;          // [ndig][2][np][N]
  const d2* gadget;  // [ndig][np] (P mod q or 0, /q)
  int np, logn;
  const d2* pq;
};

template <class X>
FENC_HD void key_combine(X& x, const KeyArgs& A) {
  x.phase([&](int t) {
    const long long N = 1LL << A.logn;
    const long long c = (long long)x.bx * x.nt + t;
    const int p = x.by % A.np, j = x.by / A.np;
    const double q = A.pq[p].x, qi = A.pq[p].y;
    const long long o = ((long long)j * A.np + p) * N + c;
    const double av = u2d(A.a[o]), ev = u2d(A.e[o]);
    const double s = u2d(A.s[(long long)p * N + c]), sp = u2d(A.sp[(long long)p * N + c]);
    const d2 g = A.gadget[(long long)j * A.np + p];
    double b = ev - mulmod(av, s, q, qi);   // key, encryption and decryption operands are words in [0, q)
    b += mulmod_c(sp, g.x, g.y, q);
    u64* k = A.key + ((long long)j * 2 * A.np + p) * N + c;
    k[0] = d2u(norm(red(b, q, qi), q));
    k[(long long)A.np * N] = A.a[o];
  });
}

// c0 = -a*s + e + m, c1 = a   (NTT form); rows: ct*nl + limb
struct EncArgs {
  const u64* a;   // [B][nl][N]
  const u64* e;   // [B][nl][N]
  const u64* m;   // [B][nl][N]
  const u64* s;   // [nprimes][N]
  u64* ct;        // [B][2][nl][N]
  int nl, logn;
  const d2* pq;
};

template <class X>
FENC_HD void enc_combine(X& x, const EncArgs& A) {
  x.phase([&](int t) {
    const long long N = 1LL << A.logn;
    const long long c = (long long)x.bx * x.nt + t;
    const int i = x.by % A.nl, b = x.by / A.nl;
    const double q = A.pq[i].x, qi = A.pq[i].y;
    const long long o = ((long long)b * A.nl + i) * N + c;
    const double av = u2d(A.a[o]);
    double r = u2d(A.e[o]) + u2d(A.m[o]) - mulmod(av, u2d(A.s[(long long)i * N + c]), q, qi);
    u64* ct = A.ct + ((long long)b * 2 * A.nl + i) * N + c;
    ct[0] = d2u(norm(red(r, q, qi), q));
    ct[(long long)A.nl * N] = A.a[o];
  });
}

// m = c0 + c1*s (NTT form); rows: ct*nl + limb
struct DecArgs {
  const u64* ct;   // [B][2][nl][N]
  const u64* s;
  u64* m;          // [B][nl][N]
  int nl, logn;
  const d2* pq;
};

template <class X>
FENC_HD void dec_combine(X& x, const DecArgs& A) {
  x.phase([&](int t) {
    const long long N = 1LL << A.logn;
    const long long c = (long long)x.bx * x.nt + t;
    const int i = x.by % A.nl, b = x.by / A.nl;
    const double q = A.pq[i].x, qi = A.pq[i].y;
    const u64* ct = A.ct + ((long long)b * 2 * A.nl + i) * N + c;
    double r = u2d(ct[0]) + mulmod(u2d(ct[(long long)A.nl * N]), u2d(A.s[(long long)i * N + c]), q, qi);
    A.m[((long long)b * A.nl + i) * N + c] = d2u(norm(red(r, q, qi), q));
  });
}

// small signed integers (one polynomial, N coefficients) reduced into limbs
struct SmallArgs {
  const long long* v;   // [B][N]
  u64* out;             // [B][nl][N]
  int nl, logn;
  const unsigned char* prime;   // [nl]
  const d2* pq;
};

template <class X>
FENC_HD void small_to_rns(X& x, const SmallArgs& A) {
  x.phase([&](int t) {
    const long long N = 1LL << A.logn;
    const long long c = (long long)x.bx * x.nt + t;
    const int l = x.by % A.nl, b = x.by / A.nl;
    const int p = A.prime[l];
    const double q = A.pq[p].x, qi = A.pq[p].y;
    const double v = (double)A.v[(long long)b * N + c];
    A.out[((long long)b * A.nl + l) * N + c] = d2u(norm(red(v, q, qi), q));
  });
}

// out = sigma_g(in) on rows of N (NTT form), or out = in*in when g == 0
struct PermArgs {
  const u64* in;
  u64* out;
  unsigned g;
  int logn;
  const unsigned char* prime;   // row -> prime (for the square)
  const d2* pq;
};

template <class X>
FENC_HD void perm_rows(X& x, const PermArgs& A) {
  x.phase([&](int t) {
    const long long N = 1LL << A.logn;
    const long long c = (long long)x.bx * x.nt + t;
    const long long r = x.by;
    if (A.g == 0) {
      const int p = A.prime[r];
      const double q = A.pq[p].x, qi = A.pq[p].y;
      const double v = u2d(A.in[r * N + c]);
      A.out[r * N + c] = d2u(norm(mulmod(v, v, q, qi), q));   // v in [0, q)
    } else {
      A.out[r * N + c] = A.in[r * N + auto_src((unsigned)c, A.g, A.logn)];
    }
  });
}

}  // namespace fk
