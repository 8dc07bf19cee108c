// Oracle method layer (fragment layout, planner, HE layers).  TEST INFRASTRUCTURE.
#pragma once
#include "orc.h"

namespace orc {

enum { KIND_FRAGMENT = 0, KIND_VECTOR = 1, KIND_TOKENS = 2 };

struct Layout {
  int kind = KIND_FRAGMENT;
  int bs = 0, c = 0, h = 0, w = 0;   // logical tensor
  int M = 0, S = 0, m = 0;           // padded side, block size, blocks per side
  int bsg = 0, cpc = 0;              // batch per ct, channels per ct (C')
  int nbg = 0, ncg = 0;              // batch groups, channel groups
  int rep = 0;                       // channels replicated across positions
  int dil = 1;                       // logical pixel (h,w) at grid (dil*h, dil*w)
  int level = 0;
  double scale = 1.0;
  int d = 0, nfeat = 0;              // vector layout: positions, features
  std::vector<int> pos;              // vector layout: feature -> position
  // KIND_TOKENS (token embeddings split into S fragments): bs tokens, c = E
  // features, S fragments of ncg ciphertexts each, d positions per token
  int n_ct() const { return kind == KIND_FRAGMENT ? nbg * ncg * S * S : kind == KIND_TOKENS ? nbg * S * ncg : nbg; }
};

// eq. (total-rot) with the convention that reproduces the optimal-S table
double rot_total_formula(double BS, double Nin, double Nout, double K, double S, double alpha);
double rot_inner_formula_eq(double Nin, double K, double S, double M, double alpha);   // eq. (inner) as printed
double optimal_S_closed_form(double K, double Nin, double Nout, double alpha, double BS);

// Token-fragment layout (Discussions, extensibility to Transformers): n tokens
// of E features, feature e in fragment e mod S at position e div S
Layout token_layout(const Context& C, int n, int E, int S, int group = 0);

Layout plan_layout(const Context& C, int bs, int c, int h, int w, int k_next, int cout_next,
                   int s_override);
Layout fragment_layout(const Context& C, int bs, int c, int h, int w, int S);
// slot positions of a logical element: returns (ct, slot) pairs (several when replicated)
void element_slots(const Layout& L, int b, int ch, int hh, int ww,
                   std::vector<std::pair<int, int>>& out);

struct Counts {
  long inner_rot = 0, outer_rot = 0, other_rot = 0, ks = 0, modup = 0, moddown = 0;
  long pmult = 0, smult = 0, rescale = 0, relin = 0;
};

std::vector<RPoly> encode_fragment(Context& C, const Layout& L, const double* x);   // x[bs][c][h][w]
std::vector<Ct> encrypt_batch(Context& C, const Layout& L, const std::vector<RPoly>& pts, u64 enc_seed);
void decrypt_decode(Context& C, const Layout& L, const std::vector<Ct>& cts, double* x);

// pt_budget: plaintext bytes under which per-position weights are materialised
// as full-scale plaintext diagonals instead of mask-basis scalar codes (the
// distinct diagonals: those of one batch group)
// only: compute just the listed output ciphertexts (and only the rotations
// their terms read), returned in the listed order.
// target: write the output straight into that layout of the output tensor
// (Arch-aware Ct Compression fused with the convolution: the repack masks
// multiply the convolution's plaintexts, its rotations merge with the outer
// rotations, one rescale); bias: bias[cout] added after the rescale
std::vector<Ct> conv2d(Context& C, const Layout& Lin, const std::vector<Ct>& in, const double* w,
                       int cout, int k, int stride, int pad, int groups, Layout& Lout, Counts& cnt,
                       long long pt_budget = 1LL << 30, int hoist = 0, const Layout* target = nullptr,
                       const double* bias = nullptr, const std::vector<int>* only = nullptr, int baby = 1);
// hoist = 1: rotated copies stay in the extended basis and each combined
// ciphertext is moved down once (see conv2d)
std::vector<Ct> avgpool2(Context& C, const Layout& Lin, const std::vector<Ct>& in, Layout& Lout,
                         Counts& cnt, int hoist = 0);
std::vector<Ct> square_act(Context& C, const Layout& Lin, const std::vector<Ct>& in, Layout& Lout,
                           Counts& cnt);
// p(x) = coeffs[0] + coeffs[1] x + ... + coeffs[d] x^d, d <= 3, one rescale per
// multiplicative level (d <= 2: one level, d = 3: two levels)
std::vector<Ct> poly_act(Context& C, const Layout& Lin, const std::vector<Ct>& in,
                         const std::vector<double>& coeffs, Layout& Lout, Counts& cnt);
// integer nearest to v (half away from zero) for |v| < 2^120, as a 128-bit integer
i128 big_code(double v);
// Repack (rot-mask-add) moves: the valid slots of source ct `src` that
// Rot(., delta) carries to target ct `dst` (Rot(z, r)[i] = z[i + r])
struct MoveGroup {
  int src = 0, dst = 0;
  long delta = 0;
  std::vector<int> src_slots;
};
std::vector<MoveGroup> repack_groups(const Context& C, const Layout& Ls, const Layout& Ld);
// a target layout of the tensor (bs, c, h, w), checked and completed
Layout check_target(const Context& C, const Layout& T, int bs, int c, int h, int w);
// the default compression target: one VECTOR ct per batch group, first fit
Layout vector_target(const Context& C, const Layout& Lin);
// Arch-aware Ct Compression into `target` (hoisted rotations per source, masks
// at q_l Delta / s_in, one ModDown per target under hoist = 1, one rescale)
std::vector<Ct> compress_to(Context& C, const Layout& Lin, const std::vector<Ct>& in, const Layout& target,
                            Layout& Lout, Counts& cnt, int hoist = 0);
std::vector<Ct> compress(Context& C, const Layout& Lin, const std::vector<Ct>& in, Layout& Lout,
                         Counts& cnt, int hoist = 0);
// only (token layouts): compute just these output cts, returned in the listed order
std::vector<Ct> fc(Context& C, const Layout& Lin, const std::vector<Ct>& in, const double* w,
                   int dout, Layout& Lout, Counts& cnt, const double* bias = nullptr,
                   const std::vector<int>* only = nullptr);
// bias[o] (channel o, or feature o of a VECTOR layout) added to every valid
// slot; out[k] is ciphertext idx[k] of L (idx null: ciphertext k)
void add_bias(const Context& C, const Layout& L, std::vector<Ct>& out, const double* bias,
              const std::vector<int>* idx = nullptr);

// scalar weight code: round half away from zero of w * scale in binary64
i64 weight_code(double w, double scale);
// split T = q_l * Delta / scale_in into a power-of-two weight scale and a mask scale
void split_scale(double T, double& dw, double& dm);

}  // namespace orc
