// Oracle method layer.  TEST INFRASTRUCTURE.
//
// What each function follows:
//   plan_layout       : Conv-aware Encoding, Alg. (fragment-packing) steps 1-3;
//                       block size by argmin of eq. (total-rot) under the
//                       slot-utilisation bound eq. (opt); Theorem 1 closed form
//                       reported beside it.
//   element_slots     : Alg. (fragment-packing) step 3b slot map, read with
//                       0-based floors: l = (i*m^2 + kappa)*BS_g + j, kappa =
//                       b_i*m + b_j, batch innermost.
//   conv2d            : eq. (multi-channel-conv) evaluated over fragment
//                       ciphertexts: inner rotations (hoisted per input ct),
//                       per-position masks and scalar weight codes, diagonal
//                       outer rotations (plain or baby-step giant-step) summed
//                       with a single ModDown, one rescale; stride by
//                       discarding fragments (Evaluation methodology,
//                       implementation paragraph).
//   avgpool2          : average pooling as a fragment sum (S >= 2) or a
//                       hoisted rotation sum (S = 1); the 1/4 is carried in
//                       the scale.
//   square_act        : x^2 polynomial activation (CMult + relinearisation).
//   poly_act          : polynomial activation of degree <= 3 (Evaluation
//                       methodology: ReLU replaced by a low-degree polynomial).
//   compress          : Arch-aware Ct Compression: rot-mask-add of sparse
//                       ciphertexts into one dense ciphertext; the mask scale is
//                       chosen so a single rescale follows (Delta1*Delta2 split).
//   fc                : diagonal matrix-vector product with baby-step
//                       giant-step (Evaluation methodology, implementation).
// Pins: tests/test_oracle_method.py (optimal-S table rotation counts, Fig. 2x2
// toy, Theorem 1 worked example, slot-map special cases S=1/BS=1 row-major and
// S=M pixel-wise, decrypted layers against a float64 numpy CNN).
#include "orc_method.h"
#include <algorithm>
#include <exception>
#include <mutex>
#include <thread>
#include <cstdlib>
#include <atomic>
#include <cmath>
#include <map>
#include <set>
#include <tuple>
#include <stdexcept>

namespace orc {

static int floordiv(int a, int b) { return (a >= 0) ? a / b : -((-a + b - 1) / b); }
static int posmod(long a, long b) { long r = a % b; return (int)(r < 0 ? r + b : r); }
static double delta_of(const Context& C) { return std::ldexp(1.0, (int)C.prm.log2scale); }

static void add_counts(Counts& a, const Counts& b) {
  a.inner_rot += b.inner_rot; a.outer_rot += b.outer_rot; a.other_rot += b.other_rot; a.ks += b.ks;
  a.modup += b.modup; a.moddown += b.moddown; a.pmult += b.pmult; a.smult += b.smult;
  a.rescale += b.rescale; a.relin += b.relin;
}

double rot_total_formula(double BS, double Nin, double Nout, double K, double S, double alpha) {
  double inner = (K > S) ? (std::pow(std::ceil(K / S), 2) - 1) * Nin : 0.0;
  double outer = std::max(alpha * S * S / BS - 1, 0.0) * Nout;
  return BS / alpha * (inner + outer);
}

double rot_inner_formula_eq(double Nin, double K, double S, double M, double alpha) {
  if (S >= M) return 0.0;
  if (K > S) return Nin / alpha * (std::pow(std::ceil(K / S), 2) - 1);
  return Nin / alpha * 4 * (S - 1) / (S * S);
}

double optimal_S_closed_form(double K, double Nin, double Nout, double alpha, double BS) {
  return std::pow(K * K * Nin * BS / (alpha * Nout), 0.25);
}

Layout fragment_layout(const Context& C, int bs, int c, int h, int w, int S) {
  Layout L;
  L.kind = KIND_FRAGMENT;
  L.bs = bs; L.c = c; L.h = h; L.w = w;
  L.M = 1;
  while (L.M < std::max(h, w)) L.M <<= 1;
  if (S < 1 || L.M % S) throw std::runtime_error("fragment_layout: S must divide M");
  L.S = S;
  L.m = L.M / S;
  const long m2 = (long)L.m * L.m;
  if (m2 > C.ns) throw std::runtime_error("fragment_layout: m^2 exceeds the slot count");
  L.bsg = (int)std::min<long>(bs, C.ns / m2);
  L.cpc = (int)(C.ns / ((long)L.bsg * m2));
  L.nbg = (bs + L.bsg - 1) / L.bsg;
  L.rep = (c < L.cpc && L.cpc % c == 0) ? 1 : 0;
  L.ncg = L.rep ? 1 : (c + L.cpc - 1) / L.cpc;
  L.dil = 1;
  L.level = C.L;
  L.scale = delta_of(C);
  return L;
}

Layout plan_layout(const Context& C, int bs, int c, int h, int w, int k_next, int cout_next,
                   int s_override) {
  int M = 1;
  while (M < std::max(h, w)) M <<= 1;
  std::vector<int> adm;
  for (int S = 1; S <= M; S <<= 1) {
    long m = M / S;
    if (m * m <= C.ns) adm.push_back(S);
  }
  if (adm.empty()) throw std::runtime_error("plan_layout: no admissible block size");
  int best = adm[0];
  if (s_override > 0) {
    if (std::find(adm.begin(), adm.end(), s_override) == adm.end())
      throw std::runtime_error("plan_layout: block size not admissible");
    best = s_override;
  } else {
    // eq. (opt): S^2 <= BS * N_in / alpha, alpha = ns / M^2  <=>  S^2 * ns <= BS * N_in * M^2
    std::vector<int> cand;
    for (int S : adm)
      if ((long double)S * S * C.ns <= (long double)bs * c * M * M) cand.push_back(S);
    if (!cand.empty()) {
      // eq. (total-rot) scaled by ns (exact integers):
      //   BS*M^2*I(K,S)*N_in + max(ns*S^2 - BS*M^2, 0)*N_out
      long double bestv = -1;
      for (int S : cand) {
        long double I = (k_next > S) ? (long double)((k_next + S - 1) / S) * ((k_next + S - 1) / S) - 1 : 0;
        long double outer = std::max<long double>((long double)C.ns * S * S - (long double)bs * M * M, 0);
        long double v = (long double)bs * M * M * I * c + outer * cout_next;
        if (bestv < 0 || v < bestv) { bestv = v; best = S; }
      }
    }
  }
  return fragment_layout(C, bs, c, h, w, best);
}

// Token embeddings split into S fragments (Discussions, extensibility to
// Transformers): the n x E input becomes n x (E/S) x S and each fragment goes
// to its own ciphertexts, so a ciphertext holds E/S features of S times more
// tokens than full-embedding packing.  Feature e lies in fragment s = e mod S
// at position p = e div S; a fragment takes ncg = ceil(ceil(E/S)/d)
// ciphertexts of d positions; slot = (p mod d) bsg + token in its group, with
// bsg tokens per ciphertext (a power of two, d bsg = N/2).
Layout token_layout(const Context& C, int n, int E, int S, int group) {
  if (n < 1 || E < 1 || S < 1 || S > E) throw std::runtime_error("token_layout: bad shape");
  const int per = (E + S - 1) / S;   // positions of the largest fragment
  int d0 = 1;
  while (d0 < per && d0 < C.ns) d0 <<= 1;
  int bsg = 1;   // tokens per ciphertext: the given grouping (a layer's output keeps its input's), or the most that fit
  if (group > 0) {
    if (group & (group - 1) || group > C.ns) throw std::runtime_error("token_layout: bad token grouping");
    bsg = group;
  } else {
    while (bsg * 2 <= n && (long)bsg * 2 * d0 <= C.ns) bsg <<= 1;
  }
  Layout L;
  L.kind = KIND_TOKENS;
  L.bs = n; L.c = E; L.h = 1; L.w = 1;
  L.M = 1; L.m = 1; L.S = S; L.cpc = 1; L.rep = 0; L.dil = 1;
  L.bsg = bsg;
  L.d = C.ns / bsg;
  L.ncg = (per + L.d - 1) / L.d;
  L.nbg = (n + bsg - 1) / bsg;
  L.nfeat = E;
  L.level = C.L;
  L.scale = delta_of(C);
  return L;
}

void element_slots(const Layout& L, int b, int ch, int hh, int ww,
                   std::vector<std::pair<int, int>>& out) {
  out.clear();
  const int bg = b / L.bsg, jb = b % L.bsg;
  if (L.kind == KIND_TOKENS) {
    const int s = ch % L.S, p = ch / L.S;
    out.push_back({(bg * L.S + s) * L.ncg + p / L.d, (p % L.d) * L.bsg + jb});
    return;
  }
  if (L.kind == KIND_VECTOR) {
    int f = (ch * L.h + hh) * L.w + ww;
    out.push_back({bg, L.pos[f] * L.bsg + jb});
    return;
  }
  const int gh = L.dil * hh, gw = L.dil * ww;
  const int u = gh % L.S, bi = gh / L.S, v = gw % L.S, bj = gw / L.S;
  auto put = [&](int cg, int q) {
    int ct = ((bg * L.ncg + cg) * L.S + u) * L.S + v;
    int slot = ((q * L.m + bi) * L.m + bj) * L.bsg + jb;
    out.push_back({ct, slot});
  };
  if (L.rep) {
    for (int q = ch; q < L.cpc; q += L.c) put(0, q);
  } else {
    put(ch / L.cpc, ch % L.cpc);
  }
}

std::vector<RPoly> encode_fragment(Context& C, const Layout& L, const double* x) {
  std::vector<std::vector<double>> z(L.n_ct(), std::vector<double>(C.ns, 0.0));
  std::vector<std::pair<int, int>> sl;
  for (int b = 0; b < L.bs; b++)
    for (int ch = 0; ch < L.c; ch++)
      for (int hh = 0; hh < L.h; hh++)
        for (int ww = 0; ww < L.w; ww++) {
          element_slots(L, b, ch, hh, ww, sl);
          double v = x[((b * L.c + ch) * L.h + hh) * L.w + ww];
          for (auto& p : sl) z[p.first][p.second] = v;
        }
  std::vector<RPoly> pts;
  for (int t = 0; t < L.n_ct(); t++) pts.push_back(encode(C, z[t], {}, L.scale, q_basis(L.level)));
  return pts;
}

std::vector<Ct> encrypt_batch(Context& C, const Layout& L, const std::vector<RPoly>& pts, u64 enc_seed) {
  std::vector<Ct> out;
  for (size_t t = 0; t < pts.size(); t++) out.push_back(encrypt(C, pts[t], L.level, L.scale, enc_seed, t));
  return out;
}

void decrypt_decode(Context& C, const Layout& L, const std::vector<Ct>& cts, double* x) {
  std::vector<std::vector<double>> z(cts.size());
  for (size_t t = 0; t < cts.size(); t++) {
    RPoly m = decrypt(C, cts[t]);
    std::vector<double> re, im;
    decode(C, m.c[0], C.primes[0], cts[t].scale, re, im);
    z[t] = re;
  }
  std::vector<std::pair<int, int>> sl;
  for (int b = 0; b < L.bs; b++)
    for (int ch = 0; ch < L.c; ch++)
      for (int hh = 0; hh < L.h; hh++)
        for (int ww = 0; ww < L.w; ww++) {
          element_slots(L, b, ch, hh, ww, sl);
          x[((b * L.c + ch) * L.h + hh) * L.w + ww] = z[sl[0].first][sl[0].second];
        }
}

// code = round half away from zero of the binary64 product w * scale (exact
// integer conversion; above 2^53 the product is already an integer)
i64 weight_code(double w, double scale) {
  double v = w * scale;
  if (!(std::fabs(v) < std::ldexp(1.0, 62))) throw std::runtime_error("weight_code: out of range");
  return (i64)std::round(v);
}

void split_scale(double T, double& dw, double& dm) {
  int e = 0;
  std::frexp(T, &e);   // T = f * 2^e, f in [0.5, 1): dw = 2^floor((e-2)/2) <= sqrt(T / 2)
  int kw = (e - 2) >> 1;
  dw = std::ldexp(1.0, kw);
  dm = T / dw;
}

static Ct zero_ct(const Context& C, int level, double scale) {
  Ct z;
  z.c0 = poly_zero(C, q_basis(level));
  z.c1 = poly_zero(C, q_basis(level));
  z.level = level;
  z.scale = scale;
  return z;
}

static void add_inplace(const Context& C, Ct& a, const Ct& b) {
  poly_add_inplace(C, a.c0, b.c0);
  poly_add_inplace(C, a.c1, b.c1);
}

struct Term { int idx; long shift; int u, v, dbi, dbj, di, dj, gi; };

// bias[o] added to every valid slot of output channel o, encoded at the
// output scale (exactly Delta) and added to c0 after the rescale
void add_bias(const Context& C, const Layout& L, std::vector<Ct>& out, const double* bias,
              const std::vector<int>* idx) {
  std::map<int, int> where;   // ciphertext index -> position in out
  for (size_t k = 0; k < out.size(); k++) where[idx ? (*idx)[k] : (int)k] = (int)k;
  std::vector<std::vector<double>> z(out.size(), std::vector<double>(C.ns, 0.0));
  std::vector<std::pair<int, int>> sl;
  for (int b = 0; b < L.bs; b++)
    for (int ch = 0; ch < L.c; ch++)
      for (int hh = 0; hh < L.h; hh++)
        for (int ww = 0; ww < L.w; ww++) {
          element_slots(L, b, ch, hh, ww, sl);
          for (auto& p : sl) {
            auto it = where.find(p.first);
            if (it != where.end())
              z[it->second][p.second] = bias[L.kind == KIND_VECTOR ? (ch * L.h + hh) * L.w + ww : ch];
          }
        }
  for (size_t t = 0; t < out.size(); t++)
    poly_add_inplace(C, out[t].c0, encode(C, z[t], {}, out[t].scale, q_basis(out[t].level)));
}

// Convolution written straight into a target layout (Arch-aware Ct
// Compression fused with the layer before it).  The natural output ct o is
// y_o = sum_r Rot(z_{o,r}, s_r) with z_{o,r} = sum_t copy_t (.) P_{o,r,t};
// the repack adds Rot(A_g (.) y_o, delta_g) into target ct d_g for every move
// group g of o.  A 0/1 mask commutes with the sum: A (.) Rot(z, s) =
// Rot(Rot(A, -s) (.) z, s), so the mask multiplies the plaintexts P (both are
// 0/1 masks or weights at the split scales Delta_w Delta_m = q_l Delta / s_in)
// and the two rotations merge into one by sigma = s_r + delta_g.  Target ct d
// is then sum_sigma Rot(Z_{d,sigma}, sigma) with one ModDown and one rescale:
// the repack adds no level and no product.  A term enters Z_{d,sigma} when its
// mask pattern meets the moved slots (zero weights included).
template <class SRC, class INCH, class PAIR>
std::vector<Ct> conv_into_target(Context& C, const Layout& Lin, const Layout& Lnat, const Layout& target,
                                 const std::vector<std::vector<Term>>& terms, int nd, int npos, bool need_mask,
                                 bool materialise, double T, double dw, double dm, SRC& source, INCH in_channel,
                                 PAIR pair_ok, const double* w, int gin, int gout, int k,
                                 const std::vector<int>& basis, int hoist, Counts& cnt) {
  const Layout Tg = check_target(C, target, Lnat.bs, Lnat.c, Lnat.h, Lnat.w);
  const std::vector<MoveGroup> mg = repack_groups(C, Lnat, Tg);
  const int S = Lin.S, m = Lin.m, bsg = Lin.bsg, cpc = Lin.cpc, lvl = Lin.level;
  const int So = Lnat.S, ncg_out = Lnat.ncg;
  // valid source pixels of a term, at channel position q (the conv's own mask)
  auto src_mask = [&](const Term& t, int q) {
    std::vector<double> z(C.ns, 0.0);
    for (int bi = 0; bi < m; bi++)
      for (int bj = 0; bj < m; bj++) {
        int gh = (bi + t.dbi) * S + t.u, gw = (bj + t.dbj) * S + t.v;
        if (gh < 0 || gh >= Lin.h || gw < 0 || gw >= Lin.w) continue;
        for (int jb = 0; jb < bsg; jb++) z[((q * m + bi) * m + bj) * bsg + jb] = 1.0;
      }
    return z;
  };
  auto wval = [&](int o, int ch, const Term& t) {
    const int grp = o / gout;
    return w[(((long long)o * gin + (ch - grp * gin)) * k + t.di) * k + t.dj];
  };
  std::map<std::pair<int, long>, Ct> Z;   // (target ct, rotation) -> diagonal sum
  auto acc_of = [&](int d, long sigma) -> Ct& {
    auto it = Z.find({d, sigma});
    if (it == Z.end()) {
      Ct z;
      z.c0 = poly_zero(C, basis);
      z.c1 = poly_zero(C, basis);
      z.level = lvl;
      z.scale = Lin.scale * T;
      it = Z.emplace(std::make_pair(d, sigma), z).first;
    }
    return it->second;
  };
  for (const MoveGroup& g : mg) {
    const int oct = g.src, go = (oct / (So * So)) % ncg_out;
    for (int r = 0; r < nd; r++) {
      const long sr = (long)r * m * m * bsg, sigma = posmod(sr + g.delta, C.ns);
      std::vector<double> ra(C.ns, 0.0);   // Rot(A_g, -s_r): the moved slots seen from z_{o,r}
      for (int sl : g.src_slots) ra[posmod((long)sl + sr, C.ns)] = 1.0;
      for (const Term& t : terms[oct]) {
        const Ct& copy = source(t.idx, t.shift);
        if (materialise) {
          std::vector<double> dz(C.ns, 0.0);
          bool any = false;
          for (int q = 0; q < npos; q++) {
            const int ch = in_channel(t.gi, q), o = go * cpc + posmod(q - r, cpc);
            if (!pair_ok(ch, o)) continue;
            const double wv = wval(o, ch, t);
            const std::vector<double> mq = src_mask(t, q);
            for (int i = 0; i < C.ns; i++)
              if (mq[i] != 0.0 && ra[i] != 0.0) {
                dz[i] = wv;
                any = true;
              }
          }
          if (!any) continue;
          add_inplace(C, acc_of(g.dst, sigma), mul_plain(C, copy, encode(C, dz, {}, T, basis), T));
          cnt.pmult++;
          continue;
        }
        for (int q = 0; q < npos; q++) {
          const int ch = in_channel(t.gi, q), o = go * cpc + posmod(q - r, cpc);
          if (!pair_ok(ch, o)) continue;
          std::vector<double> mq = need_mask ? src_mask(t, q) : std::vector<double>(C.ns, 1.0);
          bool any = false;
          for (int i = 0; i < C.ns; i++) {
            mq[i] = (mq[i] != 0.0 && ra[i] != 0.0) ? 1.0 : 0.0;
            any = any || mq[i] != 0.0;
          }
          if (!any) continue;
          Ct& acc = acc_of(g.dst, sigma);
          const i64 code = weight_code(wval(o, ch, t), dw);
          if (code == 0) continue;
          add_inplace(C, acc, mul_scalar(C, mul_plain(C, copy, encode(C, mq, {}, dm, basis), dm), code, dw));
          cnt.pmult++;
          cnt.smult++;
        }
      }
    }
  }
  std::vector<Ct> out;
  for (int d = 0; d < Tg.n_ct(); d++) {
    const Ct* z0 = nullptr;
    std::vector<const Ct*> zs;
    std::vector<i64> sh;
    for (auto& kv : Z) {
      if (kv.first.first != d) continue;
      if (hoist) {
        kv.second = mod_down_ct(C, kv.second);
        cnt.moddown++;
      }
      if (kv.first.second == 0) z0 = &kv.second;
      else {
        zs.push_back(&kv.second);
        sh.push_back(kv.first.second);
      }
    }
    Ct y;
    if (zs.empty()) {
      if (z0) y = *z0;
      else y = zero_ct(C, lvl, Lin.scale * T);
    } else {
      y = rotate_sum_lazy(C, z0, zs, sh);
      cnt.outer_rot += zs.size();
      cnt.ks += zs.size();
      cnt.modup += zs.size();
      cnt.moddown += 1;
    }
    y = rescale(C, y);
    cnt.rescale++;
    out.push_back(y);
  }
  return out;
}

std::vector<Ct> conv2d(Context& C, const Layout& Lin, const std::vector<Ct>& in, const double* w,
                       int cout, int k, int stride, int pad, int groups, Layout& Lout, Counts& cnt,
                       long long pt_budget, int hoist, const Layout* target, const double* bias,
                       const std::vector<int>* only, int baby) {
  if (Lin.kind != KIND_FRAGMENT || Lin.dil != 1) throw std::runtime_error("conv2d: needs a dense fragment layout");
  if (stride < 1 || Lin.S % stride) throw std::runtime_error("conv2d: stride must divide S");
  const int cin = Lin.c;
  if (groups < 1 || cin % groups || cout % groups) throw std::runtime_error("conv2d: bad groups");
  const int S = Lin.S, m = Lin.m, bsg = Lin.bsg, cpc = Lin.cpc, lvl = Lin.level;
  const int gin = cin / groups, gout = cout / groups;
  const double Delta = delta_of(C);
  Lout = Lin;
  Lout.c = cout;
  Lout.h = (Lin.h + 2 * pad - k) / stride + 1;
  Lout.w = (Lin.w + 2 * pad - k) / stride + 1;
  Lout.M = Lin.M / stride;
  Lout.S = S / stride;
  Lout.rep = 0;
  Lout.ncg = (cout + cpc - 1) / cpc;
  Lout.level = lvl - 1;
  Lout.scale = Delta;
  const int nd = Lin.rep ? cin : cpc;
  // Per-position masks are needed when a ciphertext holds several channel
  // positions or the kernel reads padding.  Either way T = q_l Delta / s_in is
  // split into a weight scale dw and a plaintext scale dm (Delta1 Delta2 split),
  // so weight codes stay below 2^25; without masks the plaintext is the
  // all-ones vector at dm.
  const bool need_mask = (cpc > 1) || (pad > 0);
  const double T = ((double)C.primes[lvl] * Delta) / Lin.scale;
  double dw = T, dm = 1.0;
  split_scale(T, dw, dm);
  const int npos = need_mask ? cpc : 1;

  auto in_channel = [&](int gi, int q) { return Lin.rep ? q % cin : gi * cpc + q; };
  // structural validity of the pair (input channel ch, output channel o)
  auto pair_ok = [&](int ch, int o) {
    if (ch >= cin || o >= cout) return false;
    return ch / gin == o / gout;
  };
  auto term_active = [&](int go, int gi) {
    for (int q = 0; q < npos; q++)
      for (int r = 0; r < nd; r++)
        if (pair_ok(in_channel(gi, q), go * cpc + posmod(q - r, cpc))) return true;
    return false;
  };

  // Outer rotations by baby-step giant-step (Motivation, HE multi-channel
  // convolution, which assumes BSGS): with baby step n1 the diagonal r =
  // i + n1 j contributes Rot(z_r, r s) = Rot(Rot(z_r, i s), n1 j s), and
  // Rot(c (.) P, i s) = Rot(c, i s) (.) Rot(P, i s).  So each term's copy is
  // also rotated by i s (extra hoisted rotations of the same source), its
  // plaintext is encoded rotated by i s, the products are summed into the
  // giant-step accumulator Z_j, and y = sum_j Rot(Z_j, n1 j s) takes n2 - 1
  // rotations per output instead of C' - 1.  n1 = 1 is the plain form.
  if (baby < 1) throw std::runtime_error("conv2d: baby step must be at least 1");
  if (target && baby != 1) throw std::runtime_error("conv2d: a target layout takes the plain outer rotations");
  const int n1 = std::min(baby, nd), n2 = (nd + n1 - 1) / n1;
  const long s_outer = (long)m * m * bsg;   // the slot shift between consecutive diagonals
  auto rot_vec = [&](const std::vector<double>& z, int i) {   // Rot(z, i s_outer)
    if (i == 0) return z;
    std::vector<double> r(C.ns);
    for (int x = 0; x < C.ns; x++) r[x] = z[posmod((long)x + (long)i * s_outer, C.ns)];
    return r;
  };

  const int So = Lout.S, ncg_out = Lout.ncg;
  std::vector<std::vector<Term>> terms(Lin.nbg * ncg_out * So * So);
  // the outputs computed (all, or the listed ones with only their input cone)
  std::vector<char> sel(terms.size(), only ? 0 : 1);
  if (only) {
    if (target) throw std::runtime_error("conv2d: an output subset cannot take a target layout");
    for (int o : *only) sel.at(o) = 1;
  }
  std::map<int, std::set<long>> need;
  for (int bg = 0; bg < Lin.nbg; bg++)
    for (int go = 0; go < ncg_out; go++)
      for (int uo = 0; uo < So; uo++)
        for (int vo = 0; vo < So; vo++) {
          const int oct = ((bg * ncg_out + go) * So + uo) * So + vo;
          for (int gi = 0; gi < Lin.ncg; gi++) {
            if (!term_active(go, gi)) continue;
            for (int di = 0; di < k; di++)
              for (int dj = 0; dj < k; dj++) {
                int a = uo * stride + di - pad, b = vo * stride + dj - pad;
                Term t;
                t.u = posmod(a, S); t.dbi = floordiv(a, S);
                t.v = posmod(b, S); t.dbj = floordiv(b, S);
                t.di = di; t.dj = dj; t.gi = gi;
                t.idx = ((bg * Lin.ncg + gi) * S + t.u) * S + t.v;
                t.shift = posmod(((long)t.dbi * m + t.dbj) * bsg, C.ns);
                terms[oct].push_back(t);
                if (!sel[oct]) continue;
                // baby steps i this term feeds: r = i (mod n1) for a connected (q, r)
                for (int i = 0; i < n1; i++) {
                  bool used = false;
                  for (int q = 0; q < npos && !used; q++)
                    for (int r = i; r < nd && !used; r += n1)
                      used = pair_ok(in_channel(gi, q), go * cpc + posmod(q - r, cpc));
                  const long sh = posmod(t.shift + (long)i * s_outer, C.ns);
                  if (used && sh) need[t.idx].insert(sh);
                }
              }
          }
        }
  // hoisted inner rotations: one ModUp per input ciphertext.  hoist = 1 keeps
  // the rotated copies in the extended basis Q_l U P, takes the linear
  // combination there (unrotated inputs enter as P x) and moves each combined
  // ciphertext down once; hoist = 0 moves every copy down.  Without any
  // rotated copy the combination would be P y and ModDown(P y) = y exactly,
  // so such a layer stays in Q_l either way.
  hoist = hoist && !need.empty();
  const std::vector<int> basis = hoist ? qp_basis(C, lvl) : q_basis(lvl);
  std::map<std::pair<int, long>, Ct> copies;
  {
    std::vector<std::pair<int, std::vector<i64>>> jobs;
    for (auto& kv : need) jobs.push_back({kv.first, std::vector<i64>(kv.second.begin(), kv.second.end())});
    std::vector<std::vector<Ct>> rot(jobs.size());
    par_for((int)jobs.size(), [&](int j) {
      rot[j] = hoist ? rotate_hoisted_pq(C, in[jobs[j].first], jobs[j].second)
                     : rotate_hoisted(C, in[jobs[j].first], jobs[j].second);
    });
    for (size_t j = 0; j < jobs.size(); j++) {
      const std::vector<i64>& sh = jobs[j].second;
      for (size_t i = 0; i < sh.size(); i++) copies[{jobs[j].first, sh[i]}] = rot[j][i];
      cnt.inner_rot += sh.size();
      cnt.ks += sh.size();
      cnt.modup += 1;
      if (!hoist) cnt.moddown += sh.size();
    }
  }
  std::map<int, Ct> lifted;   // P x of the unrotated inputs (hoist = 1), made before the outputs
  if (hoist) {
    std::set<int> un;
    for (size_t oct = 0; oct < terms.size(); oct++)
      if (sel[oct])
        for (const Term& t : terms[oct])
          for (int i = 0; i < n1; i++)
            if (!posmod(t.shift + (long)i * s_outer, C.ns)) un.insert(t.idx);
    std::vector<int> ul(un.begin(), un.end());
    std::vector<Ct> lv(ul.size());
    par_for((int)ul.size(), [&](int j) { lv[j] = lift_pq(C, in[ul[j]]); });
    for (size_t j = 0; j < ul.size(); j++) lifted.emplace(ul[j], lv[j]);
  }
  auto source = [&](int idx, long shift) -> const Ct& {
    if (shift) return copies.at({idx, shift});
    if (!hoist) return in[idx];
    return lifted.at(idx);
  };
  // Plaintext form: with masks, either one full-scale plaintext per (output,
  // diagonal, term) holding the weight of every position ("materialised"),
  // or a mask per (term class, position) times scalar weight codes.
  // The diagonals are the same in every batch group; the budget is charged
  // for the distinct ones, those of batch group 0.
  long long n_pt = 0;
  for (int oct = 0; oct < ncg_out * So * So; oct++) {
    const int go = (oct / (So * So)) % ncg_out;
    for (const Term& t : terms[oct])
      for (int r = 0; r < nd; r++) {
        bool any = false;
        for (int q = 0; q < npos; q++) any |= pair_ok(in_channel(t.gi, q), go * cpc + posmod(q - r, cpc));
        n_pt += any;
      }
  }
  const bool materialise = need_mask && n_pt * (lvl + 1) * (long long)C.N * 8 <= pt_budget;
  // masks: source pixel inside the logical input, restricted to position q
  std::map<std::vector<int>, RPoly> masks;
  std::mutex mask_mu;   // the cache is shared by the output threads (map nodes stay put)
  auto mask = [&](const Term& t, int q, int i) -> const RPoly& {   // rotated by i baby steps
    std::vector<int> key = {t.u, t.v, t.dbi, t.dbj, q, i};
    std::lock_guard<std::mutex> lock(mask_mu);
    auto it = masks.find(key);
    if (it != masks.end()) return it->second;
    std::vector<double> z(C.ns, 0.0);
    for (int bi = 0; bi < m; bi++)
      for (int bj = 0; bj < m; bj++) {
        int gh = (bi + t.dbi) * S + t.u, gw = (bj + t.dbj) * S + t.v;
        if (gh < 0 || gh >= Lin.h || gw < 0 || gw >= Lin.w) continue;
        for (int jb = 0; jb < bsg; jb++) z[((q * m + bi) * m + bj) * bsg + jb] = 1.0;
      }
    return masks[key] = encode(C, rot_vec(z, i), {}, dm, basis);
  };
  // the all-ones plaintext at dm: its integer polynomial is checked to be the
  // constant round(dm) (every other coefficient zero) and that constant is used
  i64 ones_c = 0;
  auto ones_const = [&]() -> i64 {
    if (ones_c) return ones_c;
    const std::vector<i64> m = encode_int(C, std::vector<double>(C.ns, 1.0), {}, dm);
    for (size_t i = 1; i < m.size(); i++)
      if (m[i] != 0) throw std::runtime_error("conv2d: all-ones plaintext is not constant");
    return ones_c = m[0];
  };

  if (target) {
    const Layout Lnat = Lout;
    std::vector<Ct> out = conv_into_target(C, Lin, Lnat, *target, terms, nd, npos, need_mask, materialise, T, dw, dm,
                                           source, in_channel, pair_ok, w, gin, gout, k, basis, hoist, cnt);
    Lout = check_target(C, *target, Lnat.bs, Lnat.c, Lnat.h, Lnat.w);
    Lout.level = lvl - 1;
    Lout.scale = Delta;
    if (bias) add_bias(C, Lout, out, bias);
    return out;
  }
  if (!materialise && !need_mask) ones_const();   // made once, before the output threads
  int n_sel = 0;
  for (char c : sel) n_sel += c;
  const bool inner = n_sel < orc_threads();   // few outputs: parallel products within each
  std::vector<Ct> out(terms.size());
  std::mutex cnt_mu;
  par_for((int)terms.size(), [&](int oct) {
          if (!sel[oct]) return;
          const int go = (oct / (So * So)) % ncg_out;
          Counts lc;
          std::vector<Ct> z(n2, zero_ct(C, lvl, Lin.scale * dw * dm));   // giant-step accumulators
          if (hoist)
            for (Ct& zr : z) {
              zr.c0 = poly_zero(C, basis);
              zr.c1 = poly_zero(C, basis);
            }
          std::vector<bool> act(n2, false);
          // The plaintext products of one output are independent: with fewer
          // outputs than threads they are made a chunk at a time in parallel
          // and added in a fixed order (sums mod q are exact either way).
          auto products = [&](int n, auto make, auto use) {
            const int chunk = inner ? orc_threads() : 1;
            std::vector<Ct> buf(chunk);
            for (int j0 = 0; j0 < n; j0 += chunk) {
              const int cn = std::min(chunk, n - j0);
              if (inner) par_for(cn, [&](int j) { buf[j] = make(j0 + j); });
              else buf[0] = make(j0);
              for (int j = 0; j < cn; j++) use(j0 + j, buf[j]);
            }
          };
          if (materialise) {
            std::vector<std::pair<const Term*, int>> tr;   // (term, diagonal) pairs with a plaintext
            std::vector<std::vector<double>> dzs;          // their diagonals, rotated by r mod n1 baby steps
            for (const Term& t : terms[oct])
              for (int r = 0; r < nd; r++) {
                std::vector<double> dz(C.ns, 0.0);
                bool any = false;
                for (int q = 0; q < npos; q++) {
                  const int ch = in_channel(t.gi, q), o = go * cpc + posmod(q - r, cpc);
                  if (!pair_ok(ch, o)) continue;
                  any = true;
                  const int grp = o / gout;
                  const double wv = w[(((long long)o * gin + (ch - grp * gin)) * k + t.di) * k + t.dj];
                  for (int bi = 0; bi < m; bi++)
                    for (int bj = 0; bj < m; bj++) {
                      int gh = (bi + t.dbi) * S + t.u, gw = (bj + t.dbj) * S + t.v;
                      if (gh < 0 || gh >= Lin.h || gw < 0 || gw >= Lin.w) continue;
                      for (int jb = 0; jb < bsg; jb++) dz[((q * m + bi) * m + bj) * bsg + jb] = wv;
                    }
                }
                if (!any) continue;
                tr.push_back({&t, r});
                dzs.push_back(rot_vec(dz, r % n1));
              }
            products(
                (int)tr.size(),
                [&](int j) {
                  const Term& t = *tr[j].first;
                  const long sh = posmod(t.shift + (long)(tr[j].second % n1) * s_outer, C.ns);
                  return mul_plain(C, source(t.idx, sh), encode(C, dzs[j], {}, T, basis), T);
                },
                [&](int j, const Ct& p) {
                  act[tr[j].second / n1] = true;
                  add_inplace(C, z[tr[j].second / n1], p);
                  lc.pmult++;
                });
          } else {
            struct TQ { const Term* t; int q, i; };   // (term, position, baby step) feeding some diagonal
            std::vector<TQ> tq;
            for (const Term& t : terms[oct])
              for (int q = 0; q < npos; q++) {
                const int ch = in_channel(t.gi, q);
                for (int i = 0; i < n1; i++) {
                  bool any = false;
                  for (int r = i; r < nd; r += n1) any |= pair_ok(ch, go * cpc + posmod(q - r, cpc));
                  if (any) tq.push_back({&t, q, i});
                }
              }
            products(
                (int)tq.size(),
                [&](int j) {
                  const Term& t = *tq[j].t;
                  const Ct& copy = source(t.idx, posmod(t.shift + (long)tq[j].i * s_outer, C.ns));
                  // the all-ones vector encodes to the constant polynomial round(dm)
                  // (also rotated): multiplying by it is multiplying by that integer
                  return need_mask ? mul_plain(C, copy, mask(t, tq[j].q, tq[j].i), dm)
                                   : mul_scalar(C, copy, ones_const(), dm);
                },
                [&](int j, const Ct& mc) {
                  const Term& t = *tq[j].t;
                  const int q = tq[j].q, ch = in_channel(t.gi, q);
                  lc.pmult++;
                  for (int r = tq[j].i; r < nd; r += n1) {
                    const int o = go * cpc + posmod(q - r, cpc);
                    if (!pair_ok(ch, o)) continue;
                    const int grp = o / gout;
                    double wv = w[(((long)o * gin + (ch - grp * gin)) * k + t.di) * k + t.dj];
                    i64 code = weight_code(wv, dw);
                    act[r / n1] = true;
                    if (code == 0) continue;
                    add_inplace(C, z[r / n1], mul_scalar(C, mc, code, dw));
                    lc.smult++;
                  }
                });
          }
          if (hoist)
            for (int j = 0; j < n2; j++)
              if (act[j]) {
                z[j] = mod_down_ct(C, z[j]);
                lc.moddown++;
              }
          std::vector<const Ct*> zs;
          std::vector<i64> sh;
          for (int j = 1; j < n2; j++)
            if (act[j]) {
              zs.push_back(&z[j]);
              sh.push_back((i64)j * n1 * s_outer);
            }
          Ct y;
          if (zs.empty()) {
            y = z[0];
          } else {
            y = rotate_sum_lazy(C, act[0] ? &z[0] : nullptr, zs, sh);
            lc.outer_rot += zs.size();
            lc.ks += zs.size();
            lc.modup += zs.size();
            lc.moddown += 1;
          }
          y = rescale(C, y);
          lc.rescale++;
          y.scale = Delta;
          out[oct] = y;
          std::lock_guard<std::mutex> lock(cnt_mu);
          add_counts(cnt, lc);
        });
  if (only) {   // the listed outputs, in the listed order
    std::vector<Ct> sub;
    for (int o : *only) sub.push_back(out[o]);
    if (bias) add_bias(C, Lout, sub, bias, only);
    return sub;
  }
  if (bias) add_bias(C, Lout, out, bias);
  return out;
}

std::vector<Ct> avgpool2(Context& C, const Layout& Lin, const std::vector<Ct>& in, Layout& Lout,
                         Counts& cnt, int hoist) {
  if (Lin.kind != KIND_FRAGMENT) throw std::runtime_error("avgpool2: needs a fragment layout");
  Lout = Lin;
  Lout.h = Lin.h / 2;
  Lout.w = Lin.w / 2;
  Lout.scale = Lin.scale * 4.0;   // the sum of four values is their mean at four times the scale
  std::vector<Ct> out;
  if (Lin.S >= 2) {
    if (Lin.dil != 1) throw std::runtime_error("avgpool2: dilated layout needs S = 1");
    const int S = Lin.S, So = S / 2;
    Lout.S = So;
    Lout.M = Lin.M / 2;
    for (int g = 0; g < Lin.nbg * Lin.ncg; g++)
      for (int uo = 0; uo < So; uo++)
        for (int vo = 0; vo < So; vo++) {
          Ct y = zero_ct(C, Lin.level, Lin.scale);
          for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) add_inplace(C, y, in[(g * S + 2 * uo + a) * S + 2 * vo + b]);
          y.scale = Lout.scale;
          out.push_back(y);
        }
  } else {
    const long d = Lin.dil, m = Lin.m, bsg = Lin.bsg;
    std::vector<i64> sh = {d * bsg, d * m * bsg, (d * m + d) * bsg};
    out.resize(in.size());
    par_for((int)in.size(), [&](int i) {
      const Ct& x = in[i];
      Ct y;
      if (hoist) {   // sum in the extended basis, one ModDown
        std::vector<Ct> r = rotate_hoisted_pq(C, x, sh);
        y = lift_pq(C, x);
        for (const Ct& t : r) add_inplace(C, y, t);
        y = mod_down_ct(C, y);
      } else {
        std::vector<Ct> r = rotate_hoisted(C, x, sh);
        y = x;
        for (const Ct& t : r) add_inplace(C, y, t);
      }
      y.scale = Lout.scale;
      out[i] = y;
    });
    const long n = (long)in.size();
    cnt.moddown += hoist ? n : 3 * n;
    cnt.other_rot += 3 * n; cnt.ks += 3 * n; cnt.modup += n;
    Lout.dil = Lin.dil * 2;
  }
  return out;
}

i128 big_code(double v) {
  if (!(std::fabs(v) < std::ldexp(1.0, 120))) throw std::runtime_error("polynomial code too large for its scale");
  return (i128)std::round(v);   // exact: |v| < 2^120 and round() returns an integral binary64
}

// Polynomial activation (Evaluation Methodology: ReLU replaced by a polynomial
// a x^2 + b x + c; the CIFAR-shaped stack uses degree 3).  Every term of one
// rescale is brought to one scale S by integer codes; the leading coefficient
// is carried by the scale itself (S = k s^2 / c) so that it is exact while the
// output scale stays within a small factor of Delta:
//   d <= 1: y = rescale(k1 x + k0),                S = Delta q_l
//   d  = 2: y = rescale(k2 x*x + k1 x + k0),       k2 = round(c2 Delta q_l / s^2), S = k2 s^2 / c2
//   d  = 3: X2 = rescale(k x*x) as for x^2;  u = k3 x' + k2' at S_u = k3 s / c3,
//           k3 = round(c3 q_{l-1} / s);  y = rescale(X2 * u + k1 x' + k0)  at S = s2 S_u
// (x' = x with its last limb dropped; k1 = round(c1 S / s), k0 = round(c0 S)).
std::vector<Ct> poly_act(Context& C, const Layout& Lin, const std::vector<Ct>& in,
                         const std::vector<double>& coeffs, Layout& Lout, Counts& cnt) {
  int d = (int)coeffs.size() - 1;
  while (d > 0 && coeffs[d] == 0.0) d--;
  if (d > 3) throw std::runtime_error("poly_act: degree above 3");
  const double s = Lin.scale, Delta = delta_of(C);
  const double c0 = coeffs.size() > 0 ? coeffs[0] : 0.0, c1 = coeffs.size() > 1 ? coeffs[1] : 0.0;
  const double c2 = coeffs.size() > 2 ? coeffs[2] : 0.0, c3 = coeffs.size() > 3 ? coeffs[3] : 0.0;
  std::vector<Ct> out;
  Lout = Lin;
  if (d <= 2) {
    if (Lin.level < 1) throw std::runtime_error("poly_act: no level left");
    const double ql = (double)C.primes[Lin.level];
    double S = Delta * ql;
    i64 k2 = 0;
    if (d == 2) {
      k2 = (i64)std::round((c2 * (Delta * ql)) / (s * s));
      if (k2 == 0) k2 = c2 > 0 ? 1 : -1;
      S = (((double)k2 * s) * s) / c2;
    }
    const i128 k1 = big_code(c1 * S / s), k0 = big_code(c0 * S);
    out.resize(in.size());
    par_for((int)in.size(), [&](int i) {
      const Ct& x = in[i];
      if (d == 2) {   // k2 x*x + k1 x + k0, relinearised and rescaled by one ModDown by P q_l
        Ct t;
        RPoly d2;
        tensor(C, x, x, k2, t.c0, t.c1, d2);
        t.level = x.level;
        t.scale = ((double)k2 * s) * s;
        out[i] = relin_rescale(C, lin_comb(C, &t, x, k1, k0), d2);
      } else {
        out[i] = rescale(C, lin_comb(C, nullptr, x, k1, k0));
      }
    });
    const long n = (long)in.size();
    if (d == 2) { cnt.relin += n; cnt.ks += n; cnt.modup += n; cnt.moddown += n; }
    cnt.rescale += n;
    Lout.level = Lin.level - 1;
    Lout.scale = S / ql;
  } else {
    if (Lin.level < 2) throw std::runtime_error("poly_act: degree 3 needs two levels");
    const double ql = (double)C.primes[Lin.level], q1 = (double)C.primes[Lin.level - 1];
    i64 k = (i64)std::round((Delta * ql) / (s * s));
    if (k < 1) k = 1;
    const double s2 = (((double)k * s) * s) / ql;
    i64 k3 = (i64)std::round((c3 * q1) / s);
    if (k3 == 0) k3 = c3 > 0 ? 1 : -1;
    const double Su = ((double)k3 * s) / c3, S = s2 * Su;
    const i128 k2c = big_code(c2 * Su), k1 = big_code(c1 * S / s), k0 = big_code(c0 * S);
    out.resize(in.size());
    par_for((int)in.size(), [&](int i) {
      const Ct& x = in[i];
      Ct t;
      RPoly d2;
      tensor(C, x, x, k, t.c0, t.c1, d2);   // X2 = k x*x at level l - 1
      t.level = x.level;
      t.scale = ((double)k * s) * s;
      const Ct X2 = relin_rescale(C, t, d2);
      const Ct xd = drop_last_limb(x);
      const Ct u = lin_comb(C, nullptr, xd, k3, k2c);
      tensor(C, X2, u, 1, t.c0, t.c1, d2);  // X2 u + k1 x' + k0 at level l - 2
      t.level = X2.level;
      t.scale = X2.scale * u.scale;
      out[i] = relin_rescale(C, lin_comb(C, &t, xd, k1, k0), d2);
    });
    const long n = (long)in.size();
    cnt.relin += 2 * n; cnt.ks += 2 * n; cnt.modup += 2 * n; cnt.moddown += 2 * n; cnt.rescale += 2 * n;
    Lout.level = Lin.level - 2;
    Lout.scale = S / q1;
  }
  for (Ct& y : out) y.scale = Lout.scale;
  return out;
}

// x^2 keeping the scale near Delta: the tensor product is multiplied by the
// integer k = round((Delta * q_l) / s^2), so (k s^2) / q_l after the rescale
std::vector<Ct> square_act(Context& C, const Layout& Lin, const std::vector<Ct>& in, Layout& Lout,
                           Counts& cnt) {
  const double s = Lin.scale, ql = (double)C.primes[Lin.level];
  i64 k = (i64)std::round((delta_of(C) * ql) / (s * s));
  if (k < 1) k = 1;
  std::vector<Ct> out(in.size());
  par_for((int)in.size(), [&](int i) {
    Ct t;
    RPoly d2;
    tensor(C, in[i], in[i], k, t.c0, t.c1, d2);
    t.level = in[i].level;
    t.scale = ((double)k * s) * s;
    out[i] = relin_rescale(C, t, d2);
  });
  const long n = (long)in.size();
  cnt.relin += n; cnt.ks += n; cnt.modup += n; cnt.moddown += n; cnt.rescale += n;
  Lout = Lin;
  Lout.level = Lin.level - 1;
  Lout.scale = (((double)k * s) * s) / ql;
  for (Ct& y : out) y.scale = Lout.scale;
  return out;
}

std::vector<MoveGroup> repack_groups(const Context& C, const Layout& Ls, const Layout& Ld) {
  if (Ls.bs != Ld.bs || Ls.c != Ld.c || Ls.h != Ld.h || Ls.w != Ld.w)
    throw std::runtime_error("repack: layouts of different tensors");
  std::map<std::tuple<int, int, long>, std::vector<int>> g;
  std::vector<std::pair<int, int>> src, dst;
  for (int b = 0; b < Ls.bs; b++)
    for (int ch = 0; ch < Ls.c; ch++)
      for (int hh = 0; hh < Ls.h; hh++)
        for (int ww = 0; ww < Ls.w; ww++) {
          element_slots(Ls, b, ch, hh, ww, src);
          element_slots(Ld, b, ch, hh, ww, dst);
          for (auto& d : dst)   // Rot(z, delta)[slot_d] = z[slot_d + delta] = z[slot_s]
            g[std::make_tuple(src[0].first, d.first, (long)posmod((long)src[0].second - d.second, C.ns))]
                .push_back(src[0].second);
        }
  std::vector<MoveGroup> out;
  for (auto& kv : g) {
    MoveGroup m;
    m.src = std::get<0>(kv.first);
    m.dst = std::get<1>(kv.first);
    m.delta = std::get<2>(kv.first);
    m.src_slots = kv.second;
    std::sort(m.src_slots.begin(), m.src_slots.end());
    out.push_back(m);
  }
  return out;
}

Layout check_target(const Context& C, const Layout& T, int bs, int c, int h, int w) {
  if (T.bs != bs || T.c != c || T.h != h || T.w != w) throw std::runtime_error("target: different tensor shape");
  if (T.kind == KIND_FRAGMENT) {
    if (T.dil != 1) throw std::runtime_error("target: dilated fragment layout");
    Layout R = fragment_layout(C, bs, c, h, w, T.S);
    if (R.M != T.M || R.m != T.m || R.bsg != T.bsg || R.cpc != T.cpc || R.nbg != T.nbg || R.ncg != T.ncg ||
        R.rep != T.rep)
      throw std::runtime_error("target: not the fragment layout of its block size");
    return R;
  }
  if (T.kind != KIND_VECTOR) throw std::runtime_error("target: unknown layout kind");
  if (T.bsg < 1 || T.d * T.bsg != C.ns || T.nbg != (bs + T.bsg - 1) / T.bsg || T.nfeat != c * h * w ||
      (int)T.pos.size() != T.nfeat)
    throw std::runtime_error("target: bad vector layout");
  std::set<int> seen(T.pos.begin(), T.pos.end());
  if ((int)seen.size() != T.nfeat || *seen.begin() < 0 || *seen.rbegin() >= T.d)
    throw std::runtime_error("target: feature positions must be distinct and below d");
  Layout R = T;
  R.cpc = 1; R.ncg = 1; R.S = 1; R.m = 1; R.M = 1; R.rep = 0; R.dil = 1;
  return R;
}

// Rot-mask-add repack into a target layout (Arch-aware Ct Compression): each
// source ciphertext is rotated once per shift it needs (hoisted: one ModUp per
// source), every rotated copy is masked to the slots that move with that
// shift, and the masked copies of one target ciphertext are summed (hoist =
// 1: in Q_l U P with one ModDown per target).  Masks are encoded at
// q_l Delta / s_in, so one rescale restores Delta.
std::vector<Ct> compress_to(Context& C, const Layout& Lin, const std::vector<Ct>& in, const Layout& target,
                            Layout& Lout, Counts& cnt, int hoist) {
  const Layout T = check_target(C, target, Lin.bs, Lin.c, Lin.h, Lin.w);
  const int lvl = Lin.level;
  if (lvl < 1) throw std::runtime_error("compress: no level left");
  const std::vector<MoveGroup> mg = repack_groups(C, Lin, T);
  std::map<int, std::set<long>> need;
  for (const MoveGroup& g : mg)
    if (g.delta) need[g.src].insert(g.delta);
  hoist = hoist && !need.empty();
  const std::vector<int> basis = hoist ? qp_basis(C, lvl) : q_basis(lvl);
  std::map<std::pair<int, long>, Ct> copies;
  {
    std::vector<std::pair<int, std::vector<i64>>> jobs;
    for (auto& kv : need) jobs.push_back({kv.first, std::vector<i64>(kv.second.begin(), kv.second.end())});
    std::vector<std::vector<Ct>> rot(jobs.size());
    par_for((int)jobs.size(), [&](int j) {
      rot[j] = hoist ? rotate_hoisted_pq(C, in[jobs[j].first], jobs[j].second)
                     : rotate_hoisted(C, in[jobs[j].first], jobs[j].second);
    });
    for (size_t j = 0; j < jobs.size(); j++) {
      const std::vector<i64>& sh = jobs[j].second;
      for (size_t i = 0; i < sh.size(); i++) copies[{jobs[j].first, sh[i]}] = rot[j][i];
      cnt.other_rot += sh.size();
      cnt.ks += sh.size();
      cnt.modup += 1;
      if (!hoist) cnt.moddown += sh.size();
    }
  }
  std::map<int, Ct> lifted;
  if (hoist)
    for (const MoveGroup& g : mg)
      if (!g.delta && !lifted.count(g.src)) lifted.emplace(g.src, lift_pq(C, in[g.src]));
  auto source = [&](int idx, long delta) -> const Ct& {
    if (delta) return copies.at({idx, delta});
    if (!hoist) return in[idx];
    return lifted.at(idx);
  };
  const double dm = ((double)C.primes[lvl] * delta_of(C)) / Lin.scale;
  Lout = T;
  Lout.level = lvl - 1;
  Lout.scale = delta_of(C);
  std::vector<Ct> out(T.n_ct());
  const bool inner = T.n_ct() < orc_threads();   // few targets: their masked copies in parallel
  par_for(T.n_ct(), [&](int d) {
    Ct acc = zero_ct(C, lvl, Lin.scale * dm);
    acc.c0 = poly_zero(C, basis);
    acc.c1 = poly_zero(C, basis);
    std::vector<const MoveGroup*> gs;
    for (const MoveGroup& g : mg)
      if (g.dst == d) gs.push_back(&g);
    std::vector<Ct> part(gs.size());
    auto masked = [&](int j) {
      const MoveGroup& g = *gs[j];
      std::vector<double> z(C.ns, 0.0);   // the moved slots after the rotation
      for (int sl : g.src_slots) z[posmod((long)sl - g.delta, C.ns)] = 1.0;
      part[j] = mul_plain(C, source(g.src, g.delta), encode(C, z, {}, dm, basis), dm);
    };
    if (inner) par_for((int)gs.size(), masked);
    else for (int j = 0; j < (int)gs.size(); j++) masked(j);
    for (const Ct& p : part) add_inplace(C, acc, p);
    if (hoist) acc = mod_down_ct(C, acc);
    Ct y = rescale(C, acc);
    y.scale = Lout.scale;
    out[d] = y;
  });
  cnt.pmult += (long)mg.size();
  if (hoist) cnt.moddown += T.n_ct();
  cnt.rescale += T.n_ct();
  return out;
}

// The library's own target when none is given: one VECTOR ciphertext per
// batch group, each source ciphertext's valid positions placed at the first
// offset where they fit (greedy first fit in ciphertext order).
Layout vector_target(const Context& C, const Layout& Lin) {
  if (Lin.kind != KIND_FRAGMENT) throw std::runtime_error("compress: needs a fragment layout");
  const int bsg = Lin.bsg, d = C.ns / bsg;
  const int per_bg = Lin.ncg * Lin.S * Lin.S;
  std::vector<std::set<int>> P(per_bg);
  std::vector<std::pair<int, int>> sl;
  for (int ch = 0; ch < Lin.c; ch++)
    for (int hh = 0; hh < Lin.h; hh++)
      for (int ww = 0; ww < Lin.w; ww++) {
        element_slots(Lin, 0, ch, hh, ww, sl);
        P[sl[0].first].insert(sl[0].second / bsg);
      }
  std::vector<char> occ(d, 0);
  std::vector<int> phi(per_bg, 0);
  for (int t = 0; t < per_bg; t++) {
    if (P[t].empty()) continue;
    int f = 0;
    for (;; f++) {
      if (*P[t].rbegin() + f >= d) throw std::runtime_error("compress: does not fit one ciphertext");
      bool ok = true;
      for (int p : P[t]) ok &= !occ[p + f];
      if (ok) break;
    }
    phi[t] = f;
    for (int p : P[t]) occ[p + f] = 1;
  }
  Layout T;
  T.kind = KIND_VECTOR;
  T.bs = Lin.bs; T.c = Lin.c; T.h = Lin.h; T.w = Lin.w;
  T.bsg = bsg; T.nbg = Lin.nbg; T.cpc = 1; T.ncg = 1; T.S = 1; T.m = 1; T.M = 1;
  T.d = d;
  T.nfeat = Lin.c * Lin.h * Lin.w;
  T.pos.resize(T.nfeat);
  for (int ch = 0; ch < Lin.c; ch++)
    for (int hh = 0; hh < Lin.h; hh++)
      for (int ww = 0; ww < Lin.w; ww++) {
        element_slots(Lin, 0, ch, hh, ww, sl);
        T.pos[(ch * Lin.h + hh) * Lin.w + ww] = sl[0].second / bsg + phi[sl[0].first];
      }
  T.level = Lin.level;
  T.scale = Lin.scale;
  return T;
}

std::vector<Ct> compress(Context& C, const Layout& Lin, const std::vector<Ct>& in, Layout& Lout,
                         Counts& cnt, int hoist) {
  return compress_to(C, Lin, in, vector_target(C, Lin), Lout, cnt, hoist);
}

// A linear layer on token fragments: every output ciphertext (fragment s',
// chunk k') is the sum over the input ciphertexts (s, k) of the diagonal
// product with the weights of the features they hold,
// W_{(s,k),(s',k')}[i][j] = w[e' = ((k' d + i) S + s')][e = ((k d + j) S + s)],
// by baby-step giant-step over d: y = sum_g Rot(sum_{(s,k), b}
// diag'_{g,b} (.) Rot(x_{s,k}, b bsg), g n1 bsg).  Baby steps are hoisted
// once per input ciphertext and shared by every output; each output sums all
// inputs before its giant steps, one lazy ModDown.
static std::vector<Ct> token_fc(Context& C, const Layout& Lin, const std::vector<Ct>& in, const double* w, int dout,
                                Layout& Lout, Counts& cnt, const double* bias, const std::vector<int>* only) {
  const int S = Lin.S, d = Lin.d, bsg = Lin.bsg, din = Lin.nfeat, lvl = Lin.level, kin = Lin.ncg;
  Lout = token_layout(C, Lin.bs, dout, S, bsg);
  Lout.level = lvl - 1;
  Lout.scale = delta_of(C);
  const int kout = Lout.ncg;
  int e = 0;
  while ((1 << e) < d) e++;
  const int n1 = 1 << ((e + 1) / 2), n2 = d / n1;
  const double dp = ((double)C.primes[lvl] * delta_of(C)) / Lin.scale;
  const int ni = S * kin, no = S * kout;   // ciphertexts per token group
  // block (input ct a = s k_in + k, output ct o = s' k_out + k'): entry [i][j]
  auto wv = [&](int a, int o, int i, int j) -> double {
    const int s = a / kin, k = a % kin, s2 = o / kout, k2 = o % kout;
    const long ein = ((long)(k * d + j)) * S + s, eout = ((long)(k2 * d + i)) * S + s2;
    if (ein >= din || eout >= dout) return 0.0;
    return w[eout * din + ein];
  };
  auto diag_active = [&](int a, int o, int kd) {
    for (int i = 0; i < d; i++)
      if (wv(a, o, i, (i + kd) % d) != 0.0) return true;
    return false;
  };
  // active (input, output, diagonal) triples; baby steps per input, giant steps per output
  std::vector<std::vector<std::vector<char>>> act(ni, std::vector<std::vector<char>>(no, std::vector<char>(d, 0)));
  par_for(ni * no, [&](int ao) {
    for (int kd = 0; kd < d; kd++) act[ao / no][ao % no][kd] = diag_active(ao / no, ao % no, kd);
  });
  std::vector<std::vector<char>> baby(ni, std::vector<char>(n1, 0)), giant(no, std::vector<char>(n2, 0));
  for (int a = 0; a < ni; a++)
    for (int o = 0; o < no; o++)
      for (int kd = 0; kd < d; kd++)
        if (act[a][o][kd]) {
          baby[a][kd % n1] = 1;
          giant[o][kd / n1] = 1;
        }
  auto plain = [&](int a, int o, int g, int b) {   // diagonal g n1 + b, rotated right by g n1 positions
    const int kd = g * n1 + b;
    std::vector<double> z(C.ns, 0.0);
    for (int l = 0; l < C.ns; l++) {
      const int i = posmod((long)l - (long)g * n1 * bsg, C.ns) / bsg;
      z[l] = wv(a, o, i, (i + kd) % d);
    }
    return encode(C, z, {}, dp, q_basis(lvl));
  };
  // outputs computed: all, or the listed ones (with only the baby steps they use)
  std::vector<char> sel(Lin.nbg * no, only ? 0 : 1);
  if (only)
    for (int t : *only) sel.at(t) = 1;
  std::vector<Ct> out(Lin.nbg * no);
  for (int bg = 0; bg < Lin.nbg; bg++) {
    std::vector<int> os;
    for (int o = 0; o < no; o++)
      if (sel[bg * no + o]) os.push_back(o);
    std::vector<std::vector<char>> need(ni, std::vector<char>(n1, 0));
    for (int a = 0; a < ni; a++)
      for (int o : os)
        for (int kd = 0; kd < d; kd++)
          if (act[a][o][kd]) need[a][kd % n1] = 1;
    // baby steps of every input ciphertext, hoisted
    std::vector<std::vector<Ct>> xr(ni);
    std::vector<std::vector<const Ct*>> xb(ni, std::vector<const Ct*>(n1, nullptr));
    par_for(ni, [&](int a) {
      std::vector<i64> bsh;
      for (int b = 1; b < n1; b++)
        if (baby[a][b] && need[a][b]) bsh.push_back((i64)b * bsg);
      if (!bsh.empty()) xr[a] = rotate_hoisted(C, in[bg * ni + a], bsh);
    });
    for (int a = 0; a < ni; a++) {
      xb[a][0] = &in[bg * ni + a];
      int j = 0;
      for (int b = 1; b < n1; b++)
        if (baby[a][b]) {
          if (need[a][b]) xb[a][b] = &xr[a][j++];
          cnt.other_rot++; cnt.ks++; cnt.moddown++;
        }
      if (n1 > 1 && std::count(baby[a].begin() + 1, baby[a].end(), 1)) cnt.modup++;
    }
    // giant-step partial sums u[o][g], each over every input and baby step
    std::vector<std::vector<Ct>> u(os.size(), std::vector<Ct>(n2, zero_ct(C, lvl, Lin.scale * dp)));
    par_for((int)os.size() * n2, [&](int t) {
      const int o = os[t / n2], g = t % n2;
      for (int a = 0; a < ni; a++)
        for (int b = 0; b < n1; b++)
          if (act[a][o][g * n1 + b]) add_inplace(C, u[t / n2][g], mul_plain(C, *xb[a][b], plain(a, o, g, b), dp));
    });
    par_for((int)os.size(), [&](int k) {
      const int o = os[k];
      std::vector<const Ct*> zs;
      std::vector<i64> sh;
      for (int g = 1; g < n2; g++)
        if (giant[o][g]) { zs.push_back(&u[k][g]); sh.push_back((i64)g * n1 * bsg); }
      Ct y = zs.empty() ? u[k][0] : rotate_sum_lazy(C, giant[o][0] ? &u[k][0] : nullptr, zs, sh);
      y.scale = Lin.scale * dp;
      y = rescale(C, y);
      y.scale = Lout.scale;
      out[bg * no + o] = y;
    });
    for (int o = 0; o < no; o++) {
      int ng = 0;
      for (int g = 1; g < n2; g++) ng += giant[o][g];
      cnt.other_rot += ng; cnt.ks += ng; cnt.modup += ng; cnt.moddown += ng ? 1 : 0; cnt.rescale++;
      for (int a = 0; a < ni; a++)
        for (int kd = 0; kd < d; kd++) cnt.pmult += act[a][o][kd];
    }
  }
  if (only) {   // the listed outputs, in the listed order
    std::vector<Ct> sub;
    for (int t : *only) sub.push_back(out[t]);
    if (bias) add_bias(C, Lout, sub, bias, only);
    return sub;
  }
  if (bias) add_bias(C, Lout, out, bias);
  return out;
}

std::vector<Ct> fc(Context& C, const Layout& Lin, const std::vector<Ct>& in, const double* w,
                   int dout, Layout& Lout, Counts& cnt, const double* bias, const std::vector<int>* only) {
  if (Lin.kind == KIND_TOKENS) return token_fc(C, Lin, in, w, dout, Lout, cnt, bias, only);
  if (only) throw std::runtime_error("fc: an output subset needs a token layout");
  if (Lin.kind != KIND_VECTOR) throw std::runtime_error("fc: needs a vector layout");
  const int d = Lin.d, bsg = Lin.bsg, din = Lin.nfeat, lvl = Lin.level;
  if (dout > d) throw std::runtime_error("fc: output larger than the vector");
  int e = 0;
  while ((1 << e) < d) e++;
  const int n1 = 1 << ((e + 1) / 2), n2 = d / n1;
  // padded d x d matrix, column = input position
  std::vector<double> Wp((size_t)d * d, 0.0);
  std::vector<char> colused(d, 0);
  for (int f = 0; f < din; f++) colused[Lin.pos[f]] = 1;
  for (int i = 0; i < dout; i++)
    for (int f = 0; f < din; f++) Wp[(size_t)i * d + Lin.pos[f]] = w[(size_t)i * din + f];
  auto diag_active = [&](int kd) {
    for (int i = 0; i < dout; i++)
      if (colused[(i + kd) % d]) return true;
    return false;
  };
  const double dp = ((double)C.primes[lvl] * delta_of(C)) / Lin.scale;
  std::vector<bool> baby(n1, false), giant(n2, false);
  for (int g = 0; g < n2; g++)
    for (int b = 0; b < n1; b++)
      if (diag_active(g * n1 + b)) { baby[b] = true; giant[g] = true; }
  // plaintext for (g, b): diag_{g n1 + b} rotated right by g*n1 slots-of-features
  std::vector<std::vector<RPoly>> pt(n2, std::vector<RPoly>(n1));
  par_for(n2 * n1, [&](int kd) {   // the diagonals are encoded independently
    const int g = kd / n1;
    if (!diag_active(kd)) return;
    std::vector<double> z(C.ns, 0.0);
    for (int l = 0; l < C.ns; l++) {
      int src = posmod((long)l - (long)g * n1 * bsg, C.ns);
      int i = src / bsg;
      z[l] = Wp[(size_t)i * d + (i + kd) % d];
    }
    pt[g][kd % n1] = encode(C, z, {}, dp, q_basis(lvl));
  });
  Lout = Layout();
  Lout.kind = KIND_VECTOR;
  Lout.bs = Lin.bs; Lout.c = dout; Lout.h = 1; Lout.w = 1;
  Lout.bsg = bsg; Lout.nbg = Lin.nbg; Lout.cpc = 1; Lout.ncg = 1; Lout.S = 1; Lout.m = 1; Lout.M = 1;
  Lout.d = d;
  Lout.nfeat = dout;
  Lout.pos.resize(dout);
  for (int i = 0; i < dout; i++) Lout.pos[i] = i;
  Lout.level = lvl - 1;
  Lout.scale = delta_of(C);
  std::vector<Ct> out;
  for (const Ct& x : in) {
    std::vector<i64> bsh;
    for (int b = 1; b < n1; b++)
      if (baby[b]) bsh.push_back((i64)b * bsg);
    std::vector<Ct> xr;
    if (!bsh.empty()) {
      xr = rotate_hoisted(C, x, bsh);
      cnt.other_rot += bsh.size(); cnt.ks += bsh.size(); cnt.modup += 1; cnt.moddown += bsh.size();
    }
    std::vector<const Ct*> xb(n1, nullptr);
    xb[0] = &x;
    for (size_t i = 0; i < bsh.size(); i++) xb[bsh[i] / bsg] = &xr[i];
    std::vector<Ct> u(n2, zero_ct(C, lvl, Lin.scale * dp));
    par_for(n2, [&](int g) {   // giant-step sums are independent
      for (int b = 0; b < n1; b++)
        if (diag_active(g * n1 + b)) add_inplace(C, u[g], mul_plain(C, *xb[b], pt[g][b], dp));
    });
    for (int kd = 0; kd < n1 * n2; kd++) cnt.pmult += diag_active(kd);
    std::vector<const Ct*> zs;
    std::vector<i64> sh;
    for (int g = 1; g < n2; g++)
      if (giant[g]) { zs.push_back(&u[g]); sh.push_back((i64)g * n1 * bsg); }
    Ct y = zs.empty() ? u[0] : rotate_sum_lazy(C, giant[0] ? &u[0] : nullptr, zs, sh);
    if (!zs.empty()) {
      y.scale = Lin.scale * dp;
      cnt.other_rot += zs.size(); cnt.ks += zs.size(); cnt.modup += zs.size(); cnt.moddown += 1;
    }
    y = rescale(C, y);
    cnt.rescale++;
    y.scale = Lout.scale;
    out.push_back(y);
  }
  if (bias) add_bias(C, Lout, out, bias);
  return out;
}

}  // namespace orc
