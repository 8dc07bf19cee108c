// Layouts, operation plans and the C ABI.
//
// Conv-aware Encoding (Alg. fragment-packing) with the readings: pad() is the
// next power of two; slot l = (i*m^2 + kappa)*BS_g + j with 0-based floors,
// kappa = b_i*m + b_j, batch innermost; a batch larger than one ciphertext
// is split into groups of BS_g = min(BS, (N/2)/m^2) images; C' = (N/2)/(BS_g
// m^2) channel positions per ciphertext, channels replicated when C < C' and
// C | C'.  Block size by argmin of eq. (total-rot) under eq. (opt).
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <map>
#include <set>
#include <unordered_set>
#include <sstream>
#include <thread>
#include <tuple>

#include "runtime.h"

using namespace fr;
using fh::mulmod;

static thread_local std::string g_err;

namespace fr {

static int next_pow2(int x) {
  int M = 1;
  while (M < x) M <<= 1;
  return M;
}

static int posmod(long long a, long long b) {
  long long r = a % b;
  return (int)(r < 0 ? r + b : r);
}

static int floordiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

Layout make_fragment(int ns, int level, double scale, int bs, int c, int h, int w, int S) {
  if (bs < 1 || c < 1 || h < 1 || w < 1) fail(FENC_EINVAL, "empty tensor");
  Layout L;
  L.kind = FENC_LAYOUT_FRAGMENT;
  L.bs = bs; L.c = c; L.h = h; L.w = w;
  L.M = next_pow2(std::max(h, w));
  if (S < 1 || L.M % S) fail(FENC_EINVAL, "block size must divide the padded side");
  L.S = S;
  L.m = L.M / S;
  const long long m2 = (long long)L.m * L.m;
  if (m2 > ns) fail(FENC_ELAYOUT, "one fragment does not fit a ciphertext (m^2 > N/2)");
  L.bsg = (int)std::min<long long>(bs, ns / m2);
  L.cpc = (int)(ns / (L.bsg * m2));
  L.nbg = (bs + L.bsg - 1) / L.bsg;
  L.rep = (c < L.cpc && L.cpc % c == 0) ? 1 : 0;
  L.ncg = L.rep ? 1 : (c + L.cpc - 1) / L.cpc;
  L.dil = 1;
  L.level = level;
  L.scale = scale;
  return L;
}

Layout plan_fragment(int ns, int level, double scale, int bs, int c, int h, int w, int k, int cout, int s_override) {
  if (bs < 1 || c < 1 || h < 1 || w < 1) fail(FENC_EINVAL, "empty tensor");
  const int M = next_pow2(std::max(h, w));
  std::vector<int> adm;
  for (int S = 1; S <= M; S <<= 1)
    if ((long long)(M / S) * (M / S) <= ns) adm.push_back(S);
  if (adm.empty()) fail(FENC_ELAYOUT, "no block size fits a ciphertext");
  int best = adm.front();
  if (s_override > 0) {
    if (std::find(adm.begin(), adm.end(), s_override) == adm.end()) fail(FENC_EINVAL, "block size not admissible");
    best = s_override;
  } else {
    __int128 bestcost = -1;
    for (int S : adm) {
      // eq. (opt): S^2 <= BS N_in / alpha with alpha = (N/2)/M^2
      if ((__int128)S * S * ns > (__int128)bs * c * M * M) continue;
      // eq. (total-rot) times N/2: BS M^2 I(K,S) N_in + max(ns S^2 - BS M^2, 0) N_out
      const __int128 ck = (k + S - 1) / S;
      const __int128 I = (k > S) ? ck * ck - 1 : 0;
      __int128 outer = (__int128)ns * S * S - (__int128)bs * M * M;
      if (outer < 0) outer = 0;
      const __int128 cost = (__int128)bs * M * M * I * c + outer * cout;
      if (bestcost < 0 || cost < bestcost) { bestcost = cost; best = S; }
    }
  }
  return make_fragment(ns, level, scale, bs, c, h, w, best);
}

// Token embeddings split into S fragments (Discussions, extensibility to
// Transformers): feature e in fragment e mod S at position e div S, tokens
// innermost; group > 0 keeps a given number of tokens per ciphertext.
Layout make_tokens(int ns, int level, double scale, int n, int E, int S, int group) {
  if (n < 1 || E < 1 || S < 1 || S > E) fail(FENC_EINVAL, "bad token tensor or fragment count");
  const int per = (E + S - 1) / S;
  int d0 = 1;
  while (d0 < per && d0 < ns) d0 <<= 1;
  int bsg = 1;
  if (group > 0) {
    if ((group & (group - 1)) || group > ns) fail(FENC_EINVAL, "tokens per ciphertext must be a power of two");
    bsg = group;
  } else {
    while (bsg * 2 <= n && (long long)bsg * 2 * d0 <= ns) bsg <<= 1;
  }
  Layout L;
  L.kind = FENC_LAYOUT_TOKENS;
  L.bs = n; L.c = E; L.h = 1; L.w = 1;
  L.M = 1; L.m = 1; L.S = S; L.cpc = 1; L.rep = 0; L.dil = 1;
  L.bsg = bsg;
  L.d = ns / bsg;
  L.ncg = (per + L.d - 1) / L.d;
  L.nbg = (n + bsg - 1) / bsg;
  L.nfeat = E;
  L.level = level;
  L.scale = scale;
  return L;
}

void layout_slots(const Layout& L, int b, int ch, int y, int x, std::vector<std::pair<int, int>>& out) {
  out.clear();
  const int bg = b / L.bsg, jb = b % L.bsg;
  if (L.kind == FENC_LAYOUT_TOKENS) {
    const int s = ch % L.S, p = ch / L.S;
    out.push_back({(bg * L.S + s) * L.ncg + p / L.d, (p % L.d) * L.bsg + jb});
    return;
  }
  if (L.kind == FENC_LAYOUT_VECTOR) {
    const int f = (ch * L.h + y) * L.w + x;
    out.push_back({bg, L.pos[f] * L.bsg + jb});
    return;
  }
  const int gy = L.dil * y, gx = L.dil * x;
  const int u = gy % L.S, bi = gy / L.S, v = gx % L.S, bj = gx / L.S;
  auto put = [&](int cg, int q) {
    out.push_back({((bg * L.ncg + cg) * L.S + u) * L.S + v, ((q * L.m + bi) * L.m + bj) * L.bsg + jb});
  };
  if (L.rep) {
    for (int q = ch; q < L.cpc; q += L.c) put(0, q);
  } else {
    put(ch / L.cpc, ch % L.cpc);
  }
}

}  // namespace fr

// ---------------------------------------------------------------- conversions
static uint64_t fnv(const void* p, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char* c = (const unsigned char*)p;
  for (size_t i = 0; i < n; i++) h = (h ^ c[i]) * 1099511628211ull;
  return h;
}

static Layout from_pub(const Ctx& C, const fenc_layout* p) {
  if (!p) fail(FENC_EINVAL, "null layout");
  Layout L;
  L.kind = p->kind; L.bs = p->bs; L.c = p->c; L.h = p->h; L.w = p->w; L.M = p->M; L.S = p->S; L.m = p->m;
  L.bsg = p->bs_g; L.cpc = p->chan_per_ct; L.nbg = p->n_bg; L.ncg = p->n_cg; L.rep = p->replicate; L.dil = p->dil;
  L.level = p->level; L.d = p->d; L.nfeat = p->n_feat; L.scale = p->scale;
  if (L.level < 0 || L.level > C.L) fail(FENC_EINVAL, "layout level out of range");
  if (L.bsg < 1 || L.nbg < 1) fail(FENC_EINVAL, "bad layout batch fields");
  if (L.kind == FENC_LAYOUT_VECTOR) {
    if (L.d * L.bsg != C.ns || L.nfeat < 1 || L.nfeat > L.d) fail(FENC_EINVAL, "bad vector layout");
    if (p->map_id == 0) {
      L.pos.resize(L.nfeat);
      for (int i = 0; i < L.nfeat; i++) L.pos[i] = i;
    } else {
      auto it = C.maps.find(p->map_id);
      if (it == C.maps.end()) fail(FENC_EINVAL, "unknown feature map");
      L.pos = it->second;
    }
  } else if (L.kind == FENC_LAYOUT_FRAGMENT) {
    if (L.S < 1 || L.m < 1 || (long long)L.m * L.m * L.bsg * L.cpc > C.ns || L.ncg < 1) fail(FENC_EINVAL, "bad fragment layout");
  } else if (L.kind == FENC_LAYOUT_TOKENS) {
    const Layout R = make_tokens(C.ns, L.level, L.scale, L.bs, L.c, L.S, L.bsg);
    if (R.d != L.d || R.ncg != L.ncg || R.nbg != L.nbg || L.h != 1 || L.w != 1 || L.nfeat != L.c)
      fail(FENC_EINVAL, "bad token layout");
  } else {
    fail(FENC_EINVAL, "unknown layout kind");
  }
  return L;
}

static fenc_layout to_pub(Ctx& C, const Layout& L) {
  fenc_layout p{};
  p.kind = L.kind; p.bs = L.bs; p.c = L.c; p.h = L.h; p.w = L.w; p.M = L.M; p.S = L.S; p.m = L.m;
  p.bs_g = L.bsg; p.chan_per_ct = L.cpc; p.n_bg = L.nbg; p.n_cg = L.ncg; p.replicate = L.rep; p.dil = L.dil;
  p.level = L.level; p.d = L.d; p.n_feat = L.nfeat; p.scale = L.scale; p.map_id = 0;
  if (L.kind == FENC_LAYOUT_VECTOR) {
    bool ident = true;
    for (int i = 0; i < L.nfeat; i++) ident &= (L.pos[i] == i);
    if (!ident) {
      uint64_t id = fnv(L.pos.data(), L.pos.size() * sizeof(int)) | 1;
      C.maps[id] = L.pos;
      p.map_id = id;
    }
  }
  return p;
}

static std::string layout_key(const Layout& L) {
  std::ostringstream o;
  o << L.kind << ',' << L.bs << ',' << L.c << ',' << L.h << ',' << L.w << ',' << L.M << ',' << L.S << ',' << L.m << ','
    << L.bsg << ',' << L.cpc << ',' << L.nbg << ',' << L.ncg << ',' << L.rep << ',' << L.dil << ',' << L.level << ','
    << L.d << ',' << L.nfeat << ',';
  o.precision(17);
  o << L.scale << ',' << (L.pos.empty() ? 0 : fnv(L.pos.data(), L.pos.size() * sizeof(int)));
  return o.str();
}

static void check_batch(const Ctx& C, const fenc_ctbatch* b, bool need_data) {
  if (!b) fail(FENC_EINVAL, "null ciphertext batch");
  if (need_data && !b->data) fail(FENC_EINVAL, "null ciphertext data");
}

// ---------------------------------------------------------------- repacking (Arch-aware Ct Compression)
// The valid slots of source ct `src` that a left rotation by `delta` carries to
// target ct `dst` (Rot(z, r)[i] = z[i + r]): the slot map between two layouts
// of one tensor, grouped by (src, dst, delta).
struct Move {
  int src = 0, dst = 0;
  long long delta = 0;
  std::vector<int> slots;
};

static std::vector<Move> repack_moves(const Ctx& C, const Layout& Ls, const Layout& Ld) {
  if (Ls.bs != Ld.bs || Ls.c != Ld.c || Ls.h != Ld.h || Ls.w != Ld.w) fail(FENC_ELAYOUT, "repack between different tensors");
  std::map<std::tuple<int, int, long long>, std::vector<int>> g;
  std::vector<std::pair<int, int>> a, b;
  for (int n = 0; n < Ls.bs; n++)
    for (int ch = 0; ch < Ls.c; ch++)
      for (int y = 0; y < Ls.h; y++)
        for (int x = 0; x < Ls.w; x++) {
          layout_slots(Ls, n, ch, y, x, a);
          layout_slots(Ld, n, ch, y, x, b);
          for (auto& d : b) g[std::make_tuple(a[0].first, d.first, (long long)posmod((long long)a[0].second - d.second, C.ns))].push_back(a[0].second);
        }
  std::vector<Move> out;
  for (auto& kv : g) {
    Move m;
    m.src = std::get<0>(kv.first);
    m.dst = std::get<1>(kv.first);
    m.delta = std::get<2>(kv.first);
    m.slots = kv.second;
    std::sort(m.slots.begin(), m.slots.end());
    out.push_back(std::move(m));
  }
  return out;
}

// A caller's target layout of tensor (bs, c, h, w): FRAGMENT layouts must be
// the Alg. fragment-packing layout of their block size, VECTOR layouts need
// distinct feature positions below d = (N/2)/bs_g.
static Layout target_layout(const Ctx& C, const Layout& T, int bs, int c, int h, int w) {
  if (T.bs != bs || T.c != c || T.h != h || T.w != w) fail(FENC_ELAYOUT, "target describes another tensor");
  if (T.kind == FENC_LAYOUT_FRAGMENT) {
    Layout R = make_fragment(C.ns, T.level, T.scale, bs, c, h, w, T.S);
    if (T.dil != 1 || R.M != T.M || R.m != T.m || R.bsg != T.bsg || R.cpc != T.cpc || R.nbg != T.nbg ||
        R.ncg != T.ncg || R.rep != T.rep)
      fail(FENC_ELAYOUT, "target is not the fragment layout of its block size");
    return R;
  }
  if (T.kind != FENC_LAYOUT_VECTOR) fail(FENC_ELAYOUT, "unknown target kind");
  if (T.bsg < 1 || T.d * T.bsg != C.ns || T.nbg != (bs + T.bsg - 1) / T.bsg || T.nfeat != c * h * w ||
      (int)T.pos.size() != T.nfeat)
    fail(FENC_ELAYOUT, "bad vector target");
  std::set<int> seen(T.pos.begin(), T.pos.end());
  if ((int)seen.size() != T.nfeat || *seen.begin() < 0 || *seen.rbegin() >= T.d)
    fail(FENC_ELAYOUT, "vector target positions must be distinct and below d");
  Layout R = T;
  R.cpc = 1; R.ncg = 1; R.S = 1; R.m = 1; R.M = 1; R.rep = 0; R.dil = 1;
  return R;
}

// Slot vectors of plaintexts, each distinct vector kept once.
struct PtSet {
  std::vector<std::vector<double>> slots;
  std::map<uint64_t, std::vector<int>> by_hash;
  int id(std::vector<double>&& z) {
    const uint64_t h = fnv(z.data(), z.size() * sizeof(double));
    auto& ids = by_hash[h];
    for (int i : ids)
      if (slots[i] == z) return i;
    ids.push_back((int)slots.size());
    slots.push_back(std::move(z));
    return (int)slots.size() - 1;
  }
};

// bias[ch] (bias[f] for VECTOR layouts) on every valid slot: out = in + B, B a
// ciphertext-shaped buffer (c1 = 0) of the encoded bias plaintexts at the
// output scale, one per distinct vector
struct BiasStage {
  GmacStage g;
  u64* B = nullptr;
  int nb = 0;
};

static BiasStage make_bias(Ctx& C, const Layout& L, const double* bias, std::vector<void*>& owner) {
  BiasStage st;
  const int n = L.n_ct(), nl = L.level + 1;
  std::vector<std::vector<double>> z(n, std::vector<double>(C.ns, 0.0));
  std::vector<std::pair<int, int>> sl;
  for (int b = 0; b < L.bs; b++)
    for (int ch = 0; ch < L.c; ch++)
      for (int y = 0; y < L.h; y++)
        for (int x = 0; x < L.w; x++) {
          layout_slots(L, b, ch, y, x, sl);
          for (auto& p : sl) z[p.first][p.second] = bias[L.kind == FENC_LAYOUT_VECTOR ? (ch * L.h + y) * L.w + x : ch];
        }
  PtSet ps;
  std::vector<int> id(n);
  for (int t = 0; t < n; t++) id[t] = ps.id(std::move(z[t]));
  st.nb = (int)ps.slots.size();
  const u64* pts = encode_plaintexts(C, ps.slots, L.scale, L.level, owner);
  std::vector<uint64_t> zero((size_t)st.nb * 2 * nl * C.N, 0);
  st.B = upload(C, zero, owner);
  for (int i = 0; i < st.nb; i++)
    fb::d2d_async(st.B + (size_t)i * 2 * nl * C.N, pts + (size_t)i * nl * C.N, (size_t)nl * C.N * 8, nullptr);
  fb::sync(nullptr);
  GmacBuild gb;
  for (int t = 0; t < n; t++) {
    gb.add_group(nullptr);
    gb.add_term(t, -1);
    gb.add_term(n + id[t], -1);
    gb.end_group();
    gb.end_output();
  }
  st.g = make_gmac(C, gb, {}, L.level, owner);
  return st;
}

static void run_bias(Ctx& C, const BiasStage& st, int level, const u64* in, u64* out, int n, fb::Stream s) {
  const long long ce = ct_elems(C, level), ps = (long long)(level + 1) * C.N;
  run_gmac(C, level + 1, st.g, in, ce, ps, n, st.B, ce, ps, out, ce, ps, s);
}

// ---------------------------------------------------------------- hoisted rotation stage
// copies[c] = Rot(in[src_c], shift_c); ModUp of each source once
struct RotStage {
  std::vector<int> src;   // ModUp'ed input cts (sorted)
  KsStage ks;
  int n = 0;
};

static RotStage make_rot_stage(Ctx& C, const std::vector<std::pair<int, long long>>& copies,
                               std::vector<void*>& owner, bool pq = false) {
  RotStage R;
  R.n = (int)copies.size();
  std::map<int, int> pos;
  for (auto& c : copies) pos[c.first] = 0;
  for (auto& kv : pos) {
    kv.second = (int)R.src.size();
    R.src.push_back(kv.first);
  }
  std::vector<std::vector<KsItem>> items;
  std::vector<fk::TailItem> tails;
  std::vector<fk::AddTerm> terms;
  for (int i = 0; i < R.n; i++) {
    const unsigned g = (unsigned)galois(C, copies[i].second);
    items.push_back({KsItem{pos[copies[i].first], g, get_key(C, g), pq ? copies[i].first : -1, copies[i].first}});
    tails.push_back(fk::TailItem{i, -1, (int)terms.size(), 1});
    terms.push_back(fk::AddTerm{copies[i].first, g});
  }
  R.ks = make_ks(C, items, tails, terms, owner);
  return R;
}

// ModUp of the listed cts (contiguous runs), then KIP/ModDown into out; with
// pq, KIP only: out[i] = (KIP_0 + P sigma(c0), KIP_1) over Q_l U P ([2][le][N])
static void run_rot_stage(Ctx& C, int level, const RotStage& R, const u64* in, u64* out, fb::Stream s,
                          bool pq = false) {
  if (R.n == 0) return;
  const int nl = level + 1, le = nl + C.K, beta = (nl + C.alpha - 1) / C.alpha;
  const long long ce = ct_elems(C, level), ee = (long long)beta * le * C.N;
  Scope sc(C.arena);
  u64* ext = (u64*)C.arena.get((size_t)R.src.size() * ee * 8, s);
  const bool copy = (long long)R.src.size() * ee * 8 <= C.own_copy;   // small stage: ext stays in cache
  for (size_t i = 0; i < R.src.size();) {
    size_t j = i;
    while (j + 1 < R.src.size() && R.src[j + 1] == R.src[j] + 1) j++;
    modup(C, level, in + R.src[i] * ce, ce, (long long)nl * C.N, (int)(j - i + 1), ext + (long long)i * ee, s, copy);
    i = j + 1;
  }
  const ExtOwn own{copy ? nullptr : in + (long long)nl * C.N, ce};
  if (pq) kip_only(C, level, ext, own, R.ks, out, in, ce, s);
  else kip_moddown(C, level, ext, own, R.ks, out, ce, nullptr, 0, in, ce, s);
}

// lazy sum stage: out[o] = base[o] + sum_r Rot(z[idx], shift), one ModDown per output
struct SumStage {
  KsStage ks;
  int nz = 0;
};

static SumStage make_sum_stage(Ctx& C, const std::vector<int>& out_idx, const std::vector<int>& base_idx,
                               const std::vector<std::vector<std::pair<int, long long>>>& terms_of,
                               std::vector<void*>& owner, int nz) {
  SumStage S;
  S.nz = nz;
  std::vector<std::vector<KsItem>> items;
  std::vector<fk::TailItem> tails;
  std::vector<fk::AddTerm> terms;
  for (size_t o = 0; o < out_idx.size(); o++) {
    std::vector<KsItem> it;
    const int off = (int)terms.size();
    for (auto& t : terms_of[o]) {
      const unsigned g = (unsigned)galois(C, t.second);
      it.push_back(KsItem{t.first, g, get_key(C, g)});
      terms.push_back(fk::AddTerm{t.first, g});
    }
    items.push_back(it);
    tails.push_back(fk::TailItem{out_idx[o], base_idx[o], off, (int)terms_of[o].size()});
  }
  S.ks = make_ks(C, items, tails, terms, owner);
  return S;
}

static void run_sum_stage(Ctx& C, int level, const SumStage& S, const u64* z, u64* out, const u64* base,
                          fb::Stream s) {
  if (S.ks.n_out == 0) return;
  const int nl = level + 1, le = nl + C.K, beta = (nl + C.alpha - 1) / C.alpha;
  const long long ce = ct_elems(C, level);
  Scope sc(C.arena);
  u64* ext = (u64*)C.arena.get((size_t)S.nz * beta * le * C.N * 8, s);
  const bool copy = (long long)S.nz * beta * le * C.N * 8 <= C.own_copy;
  modup(C, level, z, ce, (long long)nl * C.N, S.nz, ext, s, copy);
  kip_moddown(C, level, ext, ExtOwn{copy ? nullptr : z + (long long)nl * C.N, ce}, S.ks, out, ce, base, ce, z, ce,
              s);
}

// ---------------------------------------------------------------- conv2d
struct ConvPlan : Plan {
  int level = 0, n_in = 0, n_out = 0, n_zr = 0;
  int n1 = 1;        // baby step of the outer rotations (1: plain, C' - 1 rotations per output)
  bool pq = false;   // linear combinations in the extended basis, one ModDown per combined ciphertext
  RotStage rot;
  GmacStage g0, gr;
  KsStage md;        // pq: ModDown of the n_out + n_zr combined ciphertexts
  SumStage sum;
  long long n_terms = 0, n_masked = 0;
  bool has_bias = false;
  BiasStage bias;
};

// s_out > 0: the output is written in the fragment layout of the output
// tensor with block size s_out (Arch-aware Ct Compression fused with the
// convolution, see below); bias: cout values added at the output scale.
static ConvPlan* build_conv(Ctx& C, const Layout& Lin, const double* w, int cout, int k, int stride, int pad,
                            int groups, int s_out, const double* bias, bool shape_only, Layout& Lout,
                            bool pq = false, int baby = 1) {
  if (Lin.kind != FENC_LAYOUT_FRAGMENT || Lin.dil != 1) fail(FENC_ELAYOUT, "conv2d needs a dense fragment layout");
  if (k < 1 || stride < 1 || pad < 0 || cout < 1) fail(FENC_EINVAL, "bad convolution shape");
  if (Lin.S % stride) fail(FENC_EUNSUPPORTED, "stride must divide the block size");
  const int cin = Lin.c;
  if (groups < 1 || cin % groups || cout % groups) fail(FENC_EINVAL, "groups must divide both channel counts");
  if (Lin.level < 1) fail(FENC_ELEVEL, "no level left for the convolution");
  const int S = Lin.S, m = Lin.m, bsg = Lin.bsg, cpc = Lin.cpc, lvl = Lin.level;
  const int gin = cin / groups, gout = cout / groups;
  Lout = Lin;
  Lout.c = cout;
  Lout.h = (Lin.h + 2 * pad - k) / stride + 1;
  Lout.w = (Lin.w + 2 * pad - k) / stride + 1;
  if (Lout.h < 1 || Lout.w < 1) fail(FENC_EINVAL, "kernel larger than the padded input");
  Lout.M = Lin.M / stride;
  Lout.S = S / stride;
  Lout.rep = 0;
  Lout.ncg = (cout + cpc - 1) / cpc;
  Lout.level = lvl - 1;
  Lout.scale = C.Delta;
  const Layout Lnat = Lout;   // the convolution's own output layout
  const bool fused = s_out > 0;
  if (fused) Lout = make_fragment(C.ns, lvl - 1, C.Delta, Lin.bs, cout, Lnat.h, Lnat.w, s_out);
  if (shape_only) return nullptr;

  auto P = new ConvPlan;
  P->out = Lout;
  P->level = lvl;
  P->n_in = Lin.n_ct();
  P->pq = pq;
  const int nd = Lin.rep ? cin : cpc;
  // outer rotations in baby-step giant-step form (see run_conv): diagonal
  // r = i + n1 j sums into the giant-step accumulator j from copies rotated by
  // i more diagonal shifts, with plaintexts encoded rotated by as much
  const int n1 = fused ? 1 : std::max(1, std::min(baby, nd)), n2 = (nd + n1 - 1) / n1;
  const long long s_outer = (long long)m * m * bsg;
  P->n1 = n1;
  auto rot_slots = [&](std::vector<double> z, int i) {   // Rot(z, i s_outer)
    if (i == 0) return z;
    std::vector<double> r(C.ns);
    for (int x = 0; x < C.ns; x++) r[x] = z[posmod((long long)x + (long long)i * s_outer, C.ns)];
    return r;
  };
  // masks per channel position when a ciphertext holds several positions or the
  // kernel reads padding; T is always split into a weight scale dw and a
  // plaintext scale dm, so weight codes stay small (the all-ones plaintext at
  // dm when no mask is needed)
  const bool need_mask = (cpc > 1) || (pad > 0);
  const double T = ((double)C.primes[lvl] * C.Delta) / Lin.scale;
  double dw = T, dm = 1.0;
  split_scale(T, dw, dm);
  const int npos = need_mask ? cpc : 1;
  auto in_channel = [&](int gi, int q) { return Lin.rep ? q % cin : gi * cpc + q; };
  auto pair_ok = [&](int ch, int o) { return ch < cin && o < cout && ch / gin == o / gout; };
  auto term_active = [&](int go, int gi) {
    for (int q = 0; q < npos; q++)
      for (int r = 0; r < nd; r++)
        if (pair_ok(in_channel(gi, q), go * cpc + posmod(q - r, cpc))) return true;
    return false;
  };
  auto baby_used = [&](int go, int gi, int i) {   // some (q, r = i mod n1) pair connects go and gi
    for (int q = 0; q < npos; q++)
      for (int r = i; r < nd; r += n1)
        if (pair_ok(in_channel(gi, q), go * cpc + posmod(q - r, cpc))) return true;
    return false;
  };
  struct Term { int idx; long long shift; int u, v, dbi, dbj, di, dj, gi; };
  const int So = Lnat.S, ncg_out = Lnat.ncg;
  P->n_out = Lout.n_ct();
  std::vector<std::vector<Term>> terms(Lnat.n_ct());
  std::map<std::pair<int, long long>, int> copy_id;
  for (int bg = 0; bg < Lin.nbg; bg++)
    for (int go = 0; go < ncg_out; go++)
      for (int uo = 0; uo < So; uo++)
        for (int vo = 0; vo < So; vo++) {
          const int oct = ((bg * ncg_out + go) * So + uo) * So + vo;
          for (int gi = 0; gi < Lin.ncg; gi++) {
            if (!term_active(go, gi)) continue;
            for (int di = 0; di < k; di++)
              for (int dj = 0; dj < k; dj++) {
                const int a = uo * stride + di - pad, b = vo * stride + dj - pad;
                Term t;
                t.u = posmod(a, S); t.dbi = floordiv(a, S);
                t.v = posmod(b, S); t.dbj = floordiv(b, S);
                t.di = di; t.dj = dj; t.gi = gi;
                t.idx = ((bg * Lin.ncg + gi) * S + t.u) * S + t.v;
                t.shift = posmod(((long long)t.dbi * m + t.dbj) * bsg, C.ns);
                terms[oct].push_back(t);
                for (int i = 0; i < n1; i++) {
                  const long long sh = posmod(t.shift + (long long)i * s_outer, C.ns);
                  if (sh && (n1 == 1 || baby_used(go, gi, i))) copy_id[{t.idx, sh}] = 0;
                }
              }
          }
        }
  // copies ordered by shift, so rotations that share a key are adjacent
  std::vector<std::pair<int, long long>> copies;
  {
    std::vector<std::pair<long long, int>> bykey;
    for (auto& kv : copy_id) bykey.push_back({kv.first.second, kv.first.first});
    std::sort(bykey.begin(), bykey.end());
    for (auto& kv : bykey) {
      copy_id[{kv.second, kv.first}] = (int)copies.size();
      copies.push_back({kv.second, kv.first});
    }
  }
  // without rotated copies the extended basis buys nothing: the combination of
  // lifted inputs is P y and ModDown(P y) = y word for word, so the plain form
  // gives the same residues
  if (copies.empty()) P->pq = false;
  P->rot = make_rot_stage(C, copies, P->owned, P->pq);

  // Plaintext form: with masks, either one full-scale plaintext per (output,
  // diagonal, term) holding the weight of every position ("materialised"),
  // or a mask per (term class, position) times scalar weight codes.
  // The diagonals repeat in every batch group, so the budget is charged for
  // the distinct ones: those of batch group 0.
  const int out_per_bg = ncg_out * So * So;
  long long n_pt = 0;
  for (int oct = 0; oct < out_per_bg; oct++) {
    const int go = (oct / (So * So)) % ncg_out;
    for (const Term& t : terms[oct])
      for (int r = 0; r < nd; r++) {
        bool any = false;
        for (int q = 0; q < npos; q++) any = any || pair_ok(in_channel(t.gi, q), go * cpc + posmod(q - r, cpc));
        n_pt += any;
      }
  }
  const bool materialise = need_mask && n_pt * (lvl + 1) * (long long)C.N * 8 <= C.pt_budget;
  auto valid_src = [&](const Term& t, int bi, int bj) {
    const int gy = (bi + t.dbi) * S + t.u, gx = (bj + t.dbj) * S + t.v;
    return gy >= 0 && gy < Lin.h && gx >= 0 && gx < Lin.w;
  };
  // masks: source pixel inside the logical input, at channel position q; one
  // plaintext per distinct mask (away from the borders most (u, v, dbi, dbj)
  // give the same one, and their terms then share a group)
  std::map<std::vector<int>, int> mask_id;
  PtSet mset;
  auto mask_of = [&](const Term& t, int q, int i) {   // rotated by i baby steps
    std::vector<int> key = {t.u, t.v, t.dbi, t.dbj, q, i};
    auto it = mask_id.find(key);
    if (it != mask_id.end()) return it->second;
    std::vector<double> z(C.ns, 0.0);
    for (int bi = 0; bi < m; bi++)
      for (int bj = 0; bj < m; bj++) {
        if (!valid_src(t, bi, bj)) continue;
        for (int jb = 0; jb < bsg; jb++) z[((q * m + bi) * m + bj) * bsg + jb] = 1.0;
      }
    return mask_id[key] = mset.id(rot_slots(std::move(z), i));
  };
  auto ones_id = [&]() {
    const std::vector<int> key = {-1};
    auto it = mask_id.find(key);
    if (it != mask_id.end()) return it->second;
    return mask_id[key] = mset.id(std::vector<double>(C.ns, 1.0));
  };
  std::map<int64_t, int> wid;
  std::vector<int64_t> codes;
  auto weight_id = [&](int64_t code) {
    auto it = wid.find(code);
    if (it != wid.end()) return it->second;
    codes.push_back(code);
    return wid[code] = (int)codes.size() - 1;
  };
  auto wval = [&](int o, int ch, const Term& t) {
    const int grp = o / gout;
    return w[(((long long)o * gin + (ch - grp * gin)) * k + t.di) * k + t.dj];
  };
  // groups[o][r]: plaintext id -> terms (input id, weight id); plaintext ids index
  // mask_slots (mask-basis) or diag_slots (materialised, one term per group)
  typedef std::map<int, std::vector<std::pair<int, int>>> Groups;
  std::vector<std::vector<Groups>> G(fused ? 0 : P->n_out, std::vector<Groups>(n2));   // per giant step
  std::vector<std::vector<char>> act(fused ? 0 : P->n_out, std::vector<char>(n2, 0));
  std::vector<std::vector<double>> diag_slots;
  std::map<std::tuple<int, int, int>, int> diag_id;   // (output of group 0, term, diagonal) -> plaintext
  for (int oct = 0; oct < (fused ? 0 : P->n_out); oct++) {
    const int go = (oct / (So * So)) % ncg_out;
    for (size_t ti = 0; ti < terms[oct].size(); ti++) {
      const Term& t = terms[oct][ti];
      // the input of this term for baby step i; pq: unrotated inputs enter
      // lifted (P x) after the copies in the B buffer
      auto in_id_of = [&](int i) {
        const long long sh = posmod(t.shift + (long long)i * s_outer, C.ns);
        return sh ? P->n_in + copy_id.at({t.idx, sh}) : (P->pq ? P->n_in + (int)copies.size() + t.idx : t.idx);
      };
      if (materialise) {
        for (int r = 0; r < nd; r++) {
          const int in_id = in_id_of(r % n1), jg = r / n1;
          auto known = diag_id.find(std::make_tuple(oct % out_per_bg, (int)ti, r));
          if (known != diag_id.end()) {
            act[oct][jg] = 1;
            G[oct][jg][known->second].push_back({in_id, -1});
            P->n_terms++;
            continue;
          }
          std::vector<double> z;
          for (int q = 0; q < npos; q++) {
            const int ch = in_channel(t.gi, q), o = go * cpc + posmod(q - r, cpc);
            if (!pair_ok(ch, o)) continue;
            if (z.empty()) z.assign(C.ns, 0.0);
            const double wv = wval(o, ch, t);
            for (int bi = 0; bi < m; bi++)
              for (int bj = 0; bj < m; bj++) {
                if (!valid_src(t, bi, bj)) continue;
                for (int jb = 0; jb < bsg; jb++) z[((q * m + bi) * m + bj) * bsg + jb] = wv;
              }
          }
          if (z.empty()) continue;
          act[oct][jg] = 1;
          diag_id[std::make_tuple(oct % out_per_bg, (int)ti, r)] = (int)diag_slots.size();
          G[oct][jg][(int)diag_slots.size()].push_back({in_id, -1});
          diag_slots.push_back(rot_slots(std::move(z), r % n1));
          P->n_terms++;
        }
        continue;
      }
      for (int q = 0; q < npos; q++) {
        const int ch = in_channel(t.gi, q);
        for (int r = 0; r < nd; r++) {
          const int o = go * cpc + posmod(q - r, cpc);
          if (!pair_ok(ch, o)) continue;
          act[oct][r / n1] = 1;
          const int64_t code = weight_code(wval(o, ch, t), dw);   // zero codes kept: shared structure
          const int mid = need_mask ? mask_of(t, q, r % n1) : ones_id();
          G[oct][r / n1][mid].push_back({in_id_of(r % n1), weight_id(code)});
          P->n_terms++;
        }
      }
    }
  }
  // Fused repack (Arch-aware Ct Compression, one rescale for both products):
  // natural output o is y_o = sum_r Rot(z_{o,r}, s_r); the repack adds
  // Rot(A_g (.) y_o, delta_g) into target ct d_g for each move g of o.  A 0/1
  // mask commutes with the rotation sum, A (.) Rot(z, s) = Rot(Rot(A, -s) (.) z, s),
  // so A multiplies the plaintexts of z_{o,r} (masks or materialised
  // diagonals, at the convolution's own scales) and the two rotations merge:
  // target d = sum_sigma Rot(Z_{d,sigma}, sigma), sigma = s_r + delta_g, with
  // one ModDown and the layer's single rescale.  A term enters Z_{d,sigma}
  // when its mask pattern meets the moved slots (zero weights included).
  PtSet fset;
  std::map<std::pair<int, long long>, Groups> GT;
  if (fused) {
    const std::vector<Move> mv = repack_moves(C, Lnat, Lout);
    std::vector<char> ra(C.ns);
    for (const Move& g : mv) {
      const int oct = g.src, go = (oct / (So * So)) % ncg_out;
      for (int r = 0; r < nd; r++) {
        const long long sr = (long long)r * m * m * bsg, sigma = posmod(sr + g.delta, C.ns);
        std::fill(ra.begin(), ra.end(), 0);
        for (int sl : g.slots) ra[posmod(sl + sr, C.ns)] = 1;
        for (const Term& t : terms[oct]) {
          const int in_id = t.shift ? P->n_in + copy_id[{t.idx, t.shift}]
                                    : (P->pq ? P->n_in + (int)copies.size() + t.idx : t.idx);
          if (materialise) {
            std::vector<double> z(C.ns, 0.0);
            bool any = false;
            for (int q = 0; q < npos; q++) {
              const int ch = in_channel(t.gi, q), o = go * cpc + posmod(q - r, cpc);
              if (!pair_ok(ch, o)) continue;
              const double wv = wval(o, ch, t);
              for (int bi = 0; bi < m; bi++)
                for (int bj = 0; bj < m; bj++) {
                  if (!valid_src(t, bi, bj)) continue;
                  for (int jb = 0; jb < bsg; jb++) {
                    const int slot = ((q * m + bi) * m + bj) * bsg + jb;
                    if (ra[slot]) {
                      z[slot] = wv;
                      any = true;
                    }
                  }
                }
            }
            if (!any) continue;
            GT[{g.dst, sigma}][fset.id(std::move(z))].push_back({in_id, -1});
            P->n_terms++;
            continue;
          }
          for (int q = 0; q < npos; q++) {
            const int ch = in_channel(t.gi, q), o = go * cpc + posmod(q - r, cpc);
            if (!pair_ok(ch, o)) continue;
            std::vector<double> z(C.ns, 0.0);
            bool any = false;
            if (need_mask) {
              for (int bi = 0; bi < m; bi++)
                for (int bj = 0; bj < m; bj++) {
                  if (!valid_src(t, bi, bj)) continue;
                  for (int jb = 0; jb < bsg; jb++) {
                    const int slot = ((q * m + bi) * m + bj) * bsg + jb;
                    if (ra[slot]) {
                      z[slot] = 1.0;
                      any = true;
                    }
                  }
                }
            } else {
              for (int i = 0; i < C.ns; i++)
                if (ra[i]) {
                  z[i] = 1.0;
                  any = true;
                }
            }
            if (!any) continue;
            const int64_t code = weight_code(wval(o, ch, t), dw);
            GT[{g.dst, sigma}][fset.id(std::move(z))].push_back({in_id, weight_id(code)});
            P->n_terms++;
          }
        }
      }
    }
  }
  const u64* masks =
      fused ? (fset.slots.empty() ? nullptr
                                  : encode_plaintexts(C, fset.slots, materialise ? T : dm, lvl, P->owned, P->pq))
      : materialise ? (diag_slots.empty() ? nullptr : encode_plaintexts(C, diag_slots, T, lvl, P->owned, P->pq))
                    : (mset.slots.empty() ? nullptr : encode_plaintexts(C, mset.slots, dm, lvl, P->owned, P->pq));
  const long long pe = (long long)(lvl + 1 + (P->pq ? C.K : 0)) * C.N;
  GmacBuild b0, br;
  std::vector<int> sum_out, sum_base;
  std::vector<std::vector<std::pair<int, long long>>> sum_terms;
  auto emit = [&](GmacBuild& gb, const Groups& gr) {
    for (auto& kv : gr) {
      gb.add_group(kv.first < 0 ? nullptr : masks + kv.first * pe);
      if (kv.first >= 0) P->n_masked++;
      for (auto& t : kv.second) gb.add_term(t.first, t.second);
      gb.end_group();
    }
    gb.end_output();
  };
  for (int o = 0; o < (fused ? 0 : P->n_out); o++) {
    emit(b0, G[o][0]);
    std::vector<std::pair<int, long long>> tl;
    for (int j = 1; j < n2; j++)
      if (act[o][j]) {
        emit(br, G[o][j]);
        tl.push_back({P->n_zr++, (long long)j * n1 * s_outer});
      }
    if (!tl.empty()) {
      sum_out.push_back(o);
      sum_base.push_back(o);
      sum_terms.push_back(tl);
    }
  }
  for (int d = 0; d < (fused ? P->n_out : 0); d++) {
    auto z0 = GT.find({d, 0LL});
    if (z0 != GT.end()) {
      emit(b0, z0->second);
    } else {   // no unrotated part: an exact zero (one term of weight 0)
      b0.add_group(nullptr);
      b0.add_term(0, weight_id(0));
      b0.end_group();
      b0.end_output();
    }
    std::vector<std::pair<int, long long>> tl;
    for (auto it = GT.lower_bound({d, 1LL}); it != GT.end() && it->first.first == d; ++it) {
      emit(br, it->second);
      tl.push_back({P->n_zr++, it->first.second});
    }
    if (!tl.empty()) {
      sum_out.push_back(d);
      sum_base.push_back(d);
      sum_terms.push_back(tl);
    }
  }
  P->g0 = make_gmac(C, b0, codes, lvl, P->owned, P->pq, P->n_in);
  P->gr = make_gmac(C, br, codes, lvl, P->owned, P->pq, P->n_in);
  if (P->pq) P->md = make_md(C, P->n_out + P->n_zr, P->owned);
  P->sum = make_sum_stage(C, sum_out, sum_base, sum_terms, P->owned, P->n_zr);
  if (bias) {
    P->has_bias = true;
    P->bias = make_bias(C, Lout, bias, P->owned);
  }
  return P;
}

static void run_conv(Ctx& C, const ConvPlan& P, const u64* in, u64* out, fb::Stream s) {
  const int lvl = P.level, nl = lvl + 1, le = nl + C.K;
  const long long ce = ct_elems(C, lvl), ps = (long long)nl * C.N;
  Scope sc(C.arena);
  // y and the diagonals z_r share one buffer: y = yz[0, n_out), z_r = yz[n_out, ...)
  u64* yz = (u64*)C.arena.get((size_t)(P.n_out + P.n_zr) * ce * 8, s);
  u64* y = yz;
  u64* zr = yz + (long long)P.n_out * ce;
  if (P.pq) {
    const long long ee = 2LL * le * C.N, pe = (long long)le * C.N;
    u64* copies = (u64*)C.arena.get((size_t)(P.rot.n + P.n_in) * ee * 8, s);   // copies, then lifted inputs
    u64* yzp = (u64*)C.arena.get((size_t)(P.n_out + P.n_zr) * ee * 8, s);
    run_rot_stage(C, lvl, P.rot, in, copies, s, true);
    lift_to_pq(C, lvl, in, P.n_in, copies + (long long)P.rot.n * ee, s);
    run_gmac(C, nl, P.g0, in, ce, ps, P.n_in, copies, ee, pe, yzp, ee, pe, s);
    run_gmac(C, nl, P.gr, in, ce, ps, P.n_in, copies, ee, pe, yzp + (long long)P.n_out * ee, ee, pe, s);
    moddown_only(C, lvl, yzp, P.md, yz, ce, s);
  } else {
    u64* copies = (u64*)C.arena.get((size_t)std::max(1, P.rot.n) * ce * 8, s);
    run_rot_stage(C, lvl, P.rot, in, copies, s);
    run_gmac(C, nl, P.g0, in, ce, ps, P.n_in, copies, ce, ps, y, ce, ps, s);
    run_gmac(C, nl, P.gr, in, ce, ps, P.n_in, copies, ce, ps, zr, ce, ps, s);
  }
  run_sum_stage(C, lvl, P.sum, zr, y, y, s);
  if (P.has_bias) {
    u64* t = (u64*)C.arena.get((size_t)P.n_out * ct_elems(C, lvl - 1) * 8, s);
    rescale(C, lvl, y, P.n_out, t, s);
    run_bias(C, P.bias, lvl - 1, t, out, P.n_out, s);
  } else {
    rescale(C, lvl, y, P.n_out, out, s);
  }
  C.cnt.rot_inner += P.rot.n;
  C.cnt.rot_outer += P.n_zr;
  C.cnt.keyswitch += P.rot.n + P.n_zr;
  C.cnt.smult += P.n_terms;
  C.cnt.pmult += P.n_masked;
  C.cnt.cts_out += P.n_out;
}

// ---------------------------------------------------------------- avgpool
struct PoolPlan : Plan {
  int level = 0, n_in = 0, n_out = 0;
  bool pq = false;   // S = 1: rotations summed in the extended basis, one ModDown per output
  RotStage rot;
  GmacStage g;
  KsStage md;
};

static PoolPlan* build_pool(Ctx& C, const Layout& Lin, bool shape_only, Layout& Lout, bool pq = false) {
  if (Lin.kind != FENC_LAYOUT_FRAGMENT) fail(FENC_ELAYOUT, "avgpool needs a fragment layout");
  Lout = Lin;
  Lout.h = Lin.h / 2;
  Lout.w = Lin.w / 2;
  if (Lout.h < 1 || Lout.w < 1) fail(FENC_EINVAL, "input too small to pool");
  Lout.scale = Lin.scale * 4.0;
  if (Lin.S >= 2) {
    if (Lin.dil != 1) fail(FENC_ELAYOUT, "dilated layouts pool at S = 1 only");
    Lout.S = Lin.S / 2;
    Lout.M = Lin.M / 2;
  } else {
    Lout.dil = Lin.dil * 2;
  }
  if (shape_only) return nullptr;
  auto P = new PoolPlan;
  P->out = Lout;
  P->level = Lin.level;
  P->n_in = Lin.n_ct();
  P->n_out = Lout.n_ct();
  GmacBuild gb;
  if (Lin.S >= 2) {
    const int S = Lin.S, So = S / 2;
    for (int g = 0; g < Lin.nbg * Lin.ncg; g++)
      for (int uo = 0; uo < So; uo++)
        for (int vo = 0; vo < So; vo++) {
          gb.add_group(nullptr);
          for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) gb.add_term((g * S + 2 * uo + a) * S + 2 * vo + b, -1);
          gb.end_group();
          gb.end_output();
        }
  } else {
    const long long d = Lin.dil, m = Lin.m, bsg = Lin.bsg;
    const long long sh[3] = {d * bsg, d * m * bsg, (d * m + d) * bsg};
    // copies ordered by shift (rotations sharing a key are adjacent): copy i * n_in + t
    std::vector<std::pair<int, long long>> copies;
    for (int i = 0; i < 3; i++)
      for (int t = 0; t < P->n_in; t++) copies.push_back({t, sh[i] % C.ns});
    P->pq = pq;
    P->rot = make_rot_stage(C, copies, P->owned, P->pq);
    for (int t = 0; t < P->n_in; t++) {
      gb.add_group(nullptr);
      gb.add_term(P->pq ? P->n_in + 3 * P->n_in + t : t, -1);   // pq: the lifted input after the copies
      for (int i = 0; i < 3; i++) gb.add_term(P->n_in + i * P->n_in + t, -1);
      gb.end_group();
      gb.end_output();
    }
    if (P->pq) P->md = make_md(C, P->n_out, P->owned);
  }
  P->g = make_gmac(C, gb, {}, Lin.level, P->owned, P->pq, P->n_in);
  return P;
}

static void run_pool(Ctx& C, const PoolPlan& P, const u64* in, u64* out, fb::Stream s) {
  const int nl = P.level + 1, le = nl + C.K;
  const long long ce = ct_elems(C, P.level), ps = (long long)nl * C.N;
  Scope sc(C.arena);
  if (P.pq) {
    const long long ee = 2LL * le * C.N, pe = (long long)le * C.N;
    u64* copies = (u64*)C.arena.get((size_t)(P.rot.n + P.n_in) * ee * 8, s);   // copies, then lifted inputs
    u64* zp = (u64*)C.arena.get((size_t)P.n_out * ee * 8, s);
    run_rot_stage(C, P.level, P.rot, in, copies, s, true);
    lift_to_pq(C, P.level, in, P.n_in, copies + (long long)P.rot.n * ee, s);
    run_gmac(C, nl, P.g, in, ce, ps, P.n_in, copies, ee, pe, zp, ee, pe, s);
    moddown_only(C, P.level, zp, P.md, out, ce, s);
  } else {
    u64* copies = (u64*)C.arena.get((size_t)std::max(1, P.rot.n) * ce * 8, s);
    run_rot_stage(C, P.level, P.rot, in, copies, s);
    run_gmac(C, nl, P.g, in, ce, ps, P.n_in, copies, ce, ps, out, ce, ps, s);
  }
  C.cnt.rot_other += P.rot.n;
  C.cnt.keyswitch += P.rot.n;
  C.cnt.cts_out += P.n_out;
}

// ---------------------------------------------------------------- polynomial activation
// p(x) = c0 + c1 x + c2 x^2 + c3 x^3 (Evaluation methodology: ReLU replaced by a
// low-degree polynomial).  All terms of one rescale share one scale S reached
// with integer codes; the leading coefficient is carried by S itself:
//   d <= 1: rescale(k1 x + k0),                   S = Delta q_l
//   d  = 2: rescale(k2 x*x + k1 x + k0),          k2 = round(c2 Delta q_l / s^2), S = k2 s^2 / c2
//   d  = 3: X2 = rescale(k x*x) (x^2 path);  u = k3 x' + k2' at S_u = k3 s / c3 with
//           k3 = round(c3 q_{l-1} / s);  rescale(X2 * u + k1 x' + k0) at S = s2 S_u
// where x' is x without its last limb, k1 = round(c1 S / s), k0 = round(c0 S).
struct PolyPlan : Plan {
  int level = 0, n = 0, d = 0;
  bool lin = true;               // the c1 x + c0 terms are present
  KsStage ks_a, ks_b;            // relinearisation at level l and l-1
  d2 *kf = nullptr, *one = nullptr, *k1 = nullptr, *k0 = nullptr, *k3 = nullptr, *k2c = nullptr;
};

// residues of the integer nearest to v (half away from zero), |v| < 2^120
static std::vector<d2> code_residues(const Ctx& C, double v, int nl) {
  if (!(std::fabs(v) < std::ldexp(1.0, 120))) fail(FENC_ESCALE, "polynomial coefficient too large for its scale");
  const double r = std::fabs(std::round(v));
  int e = 0;
  const double f = std::frexp(r, &e);   // r = f 2^e, f in [0.5, 1)
  std::vector<d2> out(nl);
  for (int i = 0; i < nl; i++) {
    const uint64_t q = C.primes[i];
    uint64_t m;
    if (e <= 63) {
      m = (uint64_t)r % q;
    } else {   // r = mant 2^(e-53) with a 53-bit integer mantissa
      const uint64_t mant = (uint64_t)std::ldexp(f, 53);
      m = fh::mulmod(mant % q, fh::powmod(2, (uint64_t)(e - 53), q), q);
    }
    if (v < 0 && m) m = q - m;
    out[i] = cpair(m, q);
  }
  return out;
}

// t = k (a x b) over (d0, d1), d2b = its d2; with x: plus k1 x + k0, x read
// with its own strides (the same words as a when x == a); with kb1 (and x),
// b is not read but formed as kb1 x + kb0
static void run_tensor(Ctx& C, int lvl, int n, const u64* a, const u64* b, const d2* k, u64* t, u64* d2b,
                       fb::Stream s, const u64* x = nullptr, long long x_cs = 0, long long x_ps = 0,
                       const d2* k1 = nullptr, const d2* k0 = nullptr, const d2* kb1 = nullptr,
                       const d2* kb0 = nullptr) {
  const int nl = lvl + 1;
  const long long ce = ct_elems(C, lvl);
  const bool per_op = C.mode == FENC_MODE_PER_OP;
  if (kb1) b = a;   // b is formed from x; the pointer stays a valid one
  // words per limb: a (2), b unless formed or equal to a (2), x beside a (2), 3 written
  const double words = 5.0 + (b != a ? 2.0 : 0.0) + (x && x != a ? 2.0 : 0.0);
  for (int b0 = 0; b0 < n; b0 += per_op ? 1 : n) {
    const int nb = per_op ? 1 : n;
    fk::SquareArgs sa{a + b0 * ce, b + b0 * ce, t + b0 * ce, d2b + (long long)b0 * nl * C.N, nl, C.logn, ce, k, C.pq,
                      x ? x + b0 * x_cs : nullptr, x_cs, x_ps, k1, k0, kb1, kb0};
    timed(C, "tensor_square", words * nb * nl * C.N * 8, s, [&] {
      fb::tensor_square({(unsigned)std::max(1, C.N / 256), (unsigned)nl, (unsigned)nb}, std::min(256, C.N), s, sa);
    }, (a == b ? 3.0 : 4.0) * nb * nl * C.N);
    C.cnt.launches++;
  }
}

// out[b] = base[b] + k1 x[b] + k0 over nl limbs; x has its own ct / poly strides
static void run_lin(Ctx& C, int nl, int n, const u64* x, long long x_cs, long long x_ps, const u64* base, u64* out,
                    const d2* k1, const d2* k0, fb::Stream s) {
  const long long cs = 2LL * nl * C.N, ps = (long long)nl * C.N;
  const bool per_op = C.mode == FENC_MODE_PER_OP;
  for (int b0 = 0; b0 < n; b0 += per_op ? 1 : n) {
    const int nb = per_op ? 1 : n;
    fk::LinArgs la{x + b0 * x_cs, x_cs, x_ps, base ? base + b0 * cs : nullptr, cs, ps, out + b0 * cs, cs, ps,
                   nl, C.logn, k1, k0, C.pq};
    timed(C, "lin_comb", (base ? 6.0 : 4.0) * nb * nl * C.N * 8, s, [&] {
      fb::lin_comb({(unsigned)std::max(1, C.N / 256), (unsigned)(2 * nl), (unsigned)nb}, std::min(256, C.N), s, la);
    }, 2.0 * nb * nl * C.N);
    C.cnt.launches++;
  }
}

// relinearise and rescale: out (level lvl-1) = (t (d0, d1) + KS(d2b)) / q_lvl,
// by one ModDown by P q_lvl after the key inner product
static void relin_rescale(Ctx& C, int lvl, int n, const KsStage& ks, const u64* t, const u64* d2b, u64* out,
                          fb::Stream s) {
  const int nl = lvl + 1, le = nl + C.K, beta = (nl + C.alpha - 1) / C.alpha;
  Scope sc(C.arena);
  u64* ext = (u64*)C.arena.get((size_t)n * beta * le * C.N * 8, s);
  const bool copy = (long long)n * beta * le * C.N * 8 <= C.own_copy;
  modup(C, lvl, d2b, (long long)nl * C.N, 0, n, ext, s, copy);
  kip_moddown(C, lvl, ext, ExtOwn{copy ? nullptr : d2b, (long long)nl * C.N}, ks, out, ct_elems(C, lvl - 1), t,
              ct_elems(C, lvl), nullptr, 0, s, true);
  C.cnt.relin += n;
  C.cnt.keyswitch += n;
}

// The output may overwrite the input: every path reads `in` only before the
// final rescale, which reads the arena and writes `out`.
static void run_poly(Ctx& C, const PolyPlan& P, const u64* in, u64* out, fb::Stream s) {
  const int l = P.level, n = P.n;
  const long long ce = ct_elems(C, l);
  Scope sc(C.arena);
  u64* t = (u64*)C.arena.get((size_t)n * ce * 8, s);
  if (P.d <= 1) {
    run_lin(C, l + 1, n, in, ce, (long long)(l + 1) * C.N, nullptr, t, P.k1, P.k0, s);
    rescale(C, l, t, n, out, s);
  } else {
    u64* d2b = (u64*)C.arena.get((size_t)n * (l + 1) * C.N * 8, s);
    const long long xps = (long long)(l + 1) * C.N;
    if (P.d == 2) {   // k2 x*x + k1 x + k0 in one pass, then relinearised and rescaled together
      run_tensor(C, l, n, in, in, P.kf, t, d2b, s, P.lin ? in : nullptr, ce, xps, P.lin ? P.k1 : nullptr, P.k0);
      relin_rescale(C, l, n, P.ks_a, t, d2b, out, s);
    } else {
      run_tensor(C, l, n, in, in, P.kf, t, d2b, s);
      const long long c1e = ct_elems(C, l - 1);
      u64* x2 = (u64*)C.arena.get((size_t)n * c1e * 8, s);
      relin_rescale(C, l, n, P.ks_a, t, d2b, x2, s);
      // X2 u + k1 x' + k0 in one pass, with u = k3 x' + k2' formed from x' in
      // registers; x' = x without its last limb, read with level-l strides
      run_tensor(C, l - 1, n, x2, nullptr, P.one, t, d2b, s, in, ce, xps, P.lin ? P.k1 : nullptr, P.k0, P.k3,
                 P.k2c);
      relin_rescale(C, l - 1, n, P.ks_b, t, d2b, out, s);
    }
  }
  C.cnt.cts_out += n;
}

// ---------------------------------------------------------------- compress (AAC)
struct CompressPlan : Plan {
  int level = 0, n_in = 0, n_out = 0;
  bool pq = false;   // masked copies summed in the extended basis, one ModDown per target
  RotStage rot;
  GmacStage g;
  KsStage md;
};

// The library's own target when the caller gives none: one VECTOR ciphertext
// per batch group; the valid positions of each source ciphertext go to the
// first offset where they fit (greedy first fit in ciphertext order).
static Layout vector_target(const Ctx& C, const Layout& Lin) {
  if (Lin.kind != FENC_LAYOUT_FRAGMENT) fail(FENC_ELAYOUT, "compress packs fragment layouts");
  const int bsg = Lin.bsg, d = C.ns / bsg, per_bg = Lin.ncg * Lin.S * Lin.S;
  std::vector<std::set<int>> Pset(per_bg);
  std::vector<std::pair<int, int>> sl;
  for (int ch = 0; ch < Lin.c; ch++)
    for (int y = 0; y < Lin.h; y++)
      for (int x = 0; x < Lin.w; x++) {
        layout_slots(Lin, 0, ch, y, x, sl);
        Pset[sl[0].first].insert(sl[0].second / bsg);
      }
  std::vector<char> occ(d, 0);
  std::vector<int> phi(per_bg, 0);
  for (int t = 0; t < per_bg; t++) {
    if (Pset[t].empty()) continue;
    int f = 0;
    for (;; f++) {
      if (*Pset[t].rbegin() + f >= d) fail(FENC_EUNSUPPORTED, "compressed tensor does not fit one ciphertext");
      bool ok = true;
      for (int p : Pset[t]) ok = ok && !occ[p + f];
      if (ok) break;
    }
    phi[t] = f;
    for (int p : Pset[t]) occ[p + f] = 1;
  }
  Layout T;
  T.kind = FENC_LAYOUT_VECTOR;
  T.bs = Lin.bs; T.c = Lin.c; T.h = Lin.h; T.w = Lin.w;
  T.bsg = bsg; T.nbg = Lin.nbg; T.cpc = 1; T.ncg = 1; T.S = 1; T.m = 1; T.M = 1;
  T.d = d;
  T.nfeat = Lin.c * Lin.h * Lin.w;
  T.pos.resize(T.nfeat);
  for (int ch = 0; ch < Lin.c; ch++)
    for (int y = 0; y < Lin.h; y++)
      for (int x = 0; x < Lin.w; x++) {
        layout_slots(Lin, 0, ch, y, x, sl);
        T.pos[(ch * Lin.h + y) * Lin.w + x] = sl[0].second / bsg + phi[sl[0].first];
      }
  T.level = Lin.level;
  T.scale = Lin.scale;
  return T;
}

// Rot-mask-add into a target layout (Arch-aware Ct Compression without a
// preceding product to share a scale with): each source ciphertext is rotated
// once per shift it needs (hoisted: one ModUp per source), each rotated copy
// is masked to the slots that move with that shift, and the masked copies of
// a target ciphertext are summed (in Q_l U P with one ModDown per target
// under hoisting schedule 1).  Masks at q_l Delta / s_in: one rescale, one level.
static CompressPlan* build_compress(Ctx& C, const Layout& Lin, const Layout* target, bool shape_only, Layout& Lout,
                                    bool pq = false) {
  if (Lin.level < 1) fail(FENC_ELEVEL, "no level left for the compression mask");
  Lout = target ? target_layout(C, *target, Lin.bs, Lin.c, Lin.h, Lin.w) : vector_target(C, Lin);
  Lout.level = Lin.level - 1;
  Lout.scale = C.Delta;
  if (shape_only) return nullptr;
  auto P = new CompressPlan;
  P->out = Lout;
  P->level = Lin.level;
  P->n_in = Lin.n_ct();
  P->n_out = Lout.n_ct();
  const std::vector<Move> mv = repack_moves(C, Lin, Lout);
  std::map<std::pair<int, long long>, int> copy_id;
  for (const Move& g : mv)
    if (g.delta) copy_id[{g.src, g.delta}] = 0;
  std::vector<std::pair<int, long long>> copies;
  {   // copies ordered by shift, so rotations that share a key are adjacent
    std::vector<std::pair<long long, int>> bykey;
    for (auto& kv : copy_id) bykey.push_back({kv.first.second, kv.first.first});
    std::sort(bykey.begin(), bykey.end());
    for (auto& kv : bykey) {
      copy_id[{kv.second, kv.first}] = (int)copies.size();
      copies.push_back({kv.second, kv.first});
    }
  }
  P->pq = pq && !copies.empty();
  P->rot = make_rot_stage(C, copies, P->owned, P->pq);
  const double dm = ((double)C.primes[Lin.level] * C.Delta) / Lin.scale;
  PtSet ps;
  std::vector<std::vector<std::pair<int, int>>> groups(P->n_out);   // per target: (plaintext, input)
  for (const Move& g : mv) {
    std::vector<double> z(C.ns, 0.0);   // the moved slots after the rotation
    for (int sl : g.slots) z[posmod((long long)sl - g.delta, C.ns)] = 1.0;
    const int in_id = g.delta ? P->n_in + copy_id[{g.src, g.delta}]
                              : (P->pq ? P->n_in + (int)copies.size() + g.src : g.src);
    groups[g.dst].push_back({ps.id(std::move(z)), in_id});
  }
  const u64* masks = ps.slots.empty() ? nullptr : encode_plaintexts(C, ps.slots, dm, Lin.level, P->owned, P->pq);
  const long long pe = (long long)(Lin.level + 1 + (P->pq ? C.K : 0)) * C.N;
  GmacBuild gb;
  std::vector<int64_t> codes = {0};
  for (int d = 0; d < P->n_out; d++) {
    if (groups[d].empty()) {   // nothing moves here: an exact zero (one term of weight 0)
      gb.add_group(nullptr);
      gb.add_term(0, 0);
      gb.end_group();
    }
    for (auto& gt : groups[d]) {
      gb.add_group(masks + gt.first * pe);
      gb.add_term(gt.second, -1);
      gb.end_group();
    }
    gb.end_output();
  }
  P->g = make_gmac(C, gb, codes, Lin.level, P->owned, P->pq, P->n_in);
  if (P->pq) P->md = make_md(C, P->n_out, P->owned);
  return P;
}

static void run_compress(Ctx& C, const CompressPlan& P, const u64* in, u64* out, fb::Stream s) {
  const int lvl = P.level, nl = lvl + 1, le = nl + C.K;
  const long long ce = ct_elems(C, lvl), ps = (long long)nl * C.N;
  Scope sc(C.arena);
  u64* y = (u64*)C.arena.get((size_t)P.n_out * ce * 8, s);
  if (P.pq) {
    const long long ee = 2LL * le * C.N, pe = (long long)le * C.N;
    u64* copies = (u64*)C.arena.get((size_t)(P.rot.n + P.n_in) * ee * 8, s);   // copies, then lifted inputs
    u64* yp = (u64*)C.arena.get((size_t)P.n_out * ee * 8, s);
    run_rot_stage(C, lvl, P.rot, in, copies, s, true);
    lift_to_pq(C, lvl, in, P.n_in, copies + (long long)P.rot.n * ee, s);
    run_gmac(C, nl, P.g, in, ce, ps, P.n_in, copies, ee, pe, yp, ee, pe, s);
    moddown_only(C, lvl, yp, P.md, y, ce, s);
  } else {
    u64* copies = (u64*)C.arena.get((size_t)std::max(1, P.rot.n) * ce * 8, s);
    run_rot_stage(C, lvl, P.rot, in, copies, s);
    run_gmac(C, nl, P.g, in, ce, ps, P.n_in, copies, ce, ps, y, ce, ps, s);
  }
  rescale(C, lvl, y, P.n_out, out, s);
  C.cnt.rot_other += P.rot.n;
  C.cnt.keyswitch += P.rot.n;
  C.cnt.pmult += P.g.n_masked;
  C.cnt.cts_out += P.n_out;
}

// ---------------------------------------------------------------- fc (diagonal BSGS)
struct FcPlan : Plan {
  int level = 0, n_in = 0, n_out = 0, n_zr = 0;
  RotStage rot;
  GmacStage g0, gr;
  SumStage sum;
  bool has_bias = false;
  BiasStage bias;
};

// A linear layer on token fragments (Discussions, extensibility to
// Transformers).  Each output ciphertext (fragment s', chunk k') sums, over the
// input ciphertexts (s, k) of its token group, the diagonal products with the
// weights of the features they hold, W[i][j] = w[e' = (k' d + i) S + s'][e =
// (k d + j) S + s], by baby-step giant-step over the d positions:
// y = sum_g Rot(sum_{(s,k), b} diag'_{g,b} (.) Rot(x_{s,k}, b bs_g), g n1 bs_g).
// Baby steps are hoisted once per input ciphertext and shared by every
// output; each output sums all its inputs before one lazy giant-step sum.  A
// diagonal is live when some weight on it is nonzero.
static FcPlan* build_fc_tokens(Ctx& C, const Layout& Lin, const double* W, int dout, const double* bias,
                               bool shape_only, Layout& Lout) {
  if (Lin.level < 1) fail(FENC_ELEVEL, "no level left for the fc layer");
  const int S = Lin.S, d = Lin.d, bsg = Lin.bsg, din = Lin.nfeat, lvl = Lin.level, kin = Lin.ncg;
  if (dout < 1) fail(FENC_EINVAL, "fc without outputs");
  Lout = make_tokens(C.ns, lvl - 1, C.Delta, Lin.bs, dout, S, bsg);
  if (shape_only) return nullptr;
  const int kout = Lout.ncg, ni = S * kin, no = S * kout;
  int e = 0;
  while ((1 << e) < d) e++;
  const int n1 = 1 << ((e + 1) / 2), n2 = d / n1;
  auto wv = [&](int a, int o, int i, int j) -> double {   // block (input ct a, output ct o), entry [i][j]
    const int s = a / kin, k = a % kin, s2 = o / kout, k2 = o % kout;
    const long long ein = ((long long)k * d + j) * S + s, eout = ((long long)k2 * d + i) * S + s2;
    return ein < din && eout < dout ? W[eout * din + ein] : 0.0;
  };
  std::vector<char> act((size_t)ni * no * d, 0);
  auto live = [&](int a, int o, int kd) -> char& { return act[((size_t)a * no + o) * d + kd]; };
  std::vector<std::vector<char>> baby(ni, std::vector<char>(n1, 0)), giant(no, std::vector<char>(n2, 0));
  for (int a = 0; a < ni; a++)
    for (int o = 0; o < no; o++)
      for (int kd = 0; kd < d; kd++) {
        for (int i = 0; i < d && !live(a, o, kd); i++) live(a, o, kd) = wv(a, o, i, (i + kd) % d) != 0.0;
        if (live(a, o, kd)) {
          baby[a][kd % n1] = 1;
          giant[o][kd / n1] = 1;
        }
      }
  auto P = new FcPlan;
  P->out = Lout;
  P->level = lvl;
  P->n_in = Lin.n_ct();
  P->n_out = Lout.n_ct();
  const double dp = ((double)C.primes[lvl] * C.Delta) / Lin.scale;
  std::vector<std::vector<double>> slots;
  std::vector<int> pid((size_t)ni * no * d, -1);
  for (int a = 0; a < ni; a++)
    for (int o = 0; o < no; o++)
      for (int kd = 0; kd < d; kd++) {
        if (!live(a, o, kd)) continue;
        const int g = kd / n1;
        std::vector<double> z(C.ns);
        for (int l = 0; l < C.ns; l++) {
          const int i = posmod((long long)l - (long long)g * n1 * bsg, C.ns) / bsg;
          z[l] = wv(a, o, i, (i + kd) % d);
        }
        pid[((size_t)a * no + o) * d + kd] = (int)slots.size();
        slots.push_back(std::move(z));
      }
  const u64* pts = encode_plaintexts(C, slots, dp, lvl, P->owned);
  const long long pe = (long long)(lvl + 1) * C.N;
  // baby copies of every input ciphertext, ordered by shift so rotations sharing a key are adjacent
  std::vector<std::pair<int, long long>> copies;
  std::map<std::pair<int, int>, int> copy_of;   // (input ct, baby step) -> copy
  for (int b = 1; b < n1; b++)
    for (int t = 0; t < P->n_in; t++)
      if (baby[t % ni][b]) {
        copy_of[{t, b}] = (int)copies.size();
        copies.push_back({t, (long long)b * bsg});
      }
  P->rot = make_rot_stage(C, copies, P->owned);
  GmacBuild b0, br;
  std::vector<int> so, sb;
  std::vector<std::vector<std::pair<int, long long>>> st;
  for (int bg = 0; bg < Lin.nbg; bg++)
    for (int o = 0; o < no; o++) {
      const int oid = bg * no + o;
      std::vector<std::pair<int, long long>> tl;
      for (int g = 0; g < n2; g++) {
        if (g > 0 && !giant[o][g]) continue;
        GmacBuild& gb = g == 0 ? b0 : br;
        for (int a = 0; a < ni; a++)
          for (int b = 0; b < n1; b++) {
            const int id = pid[((size_t)a * no + o) * d + g * n1 + b];
            if (id < 0) continue;
            const int t = bg * ni + a;
            gb.add_group(pts + id * pe);
            gb.add_term(b == 0 ? t : P->n_in + copy_of.at({t, b}), -1);
            gb.end_group();
          }
        gb.end_output();
        if (g > 0) tl.push_back({P->n_zr++, (long long)g * n1 * bsg});
      }
      if (!tl.empty()) {
        so.push_back(oid);
        sb.push_back(oid);
        st.push_back(tl);
      }
    }
  P->g0 = make_gmac(C, b0, {}, lvl, P->owned);
  P->gr = make_gmac(C, br, {}, lvl, P->owned);
  P->sum = make_sum_stage(C, so, sb, st, P->owned, P->n_zr);
  if (bias) {
    P->has_bias = true;
    P->bias = make_bias(C, Lout, bias, P->owned);
  }
  return P;
}

static FcPlan* build_fc(Ctx& C, const Layout& Lin, const double* W, int dout, const double* bias, bool shape_only,
                        Layout& Lout) {
  if (Lin.kind == FENC_LAYOUT_TOKENS) return build_fc_tokens(C, Lin, W, dout, bias, shape_only, Lout);
  if (Lin.kind != FENC_LAYOUT_VECTOR) fail(FENC_ELAYOUT, "fc needs a vector layout");
  if (Lin.level < 1) fail(FENC_ELEVEL, "no level left for the fc layer");
  const int d = Lin.d, bsg = Lin.bsg, din = Lin.nfeat, lvl = Lin.level;
  if (dout < 1 || dout > d) fail(FENC_EINVAL, "fc output larger than the vector");
  Lout = Layout();
  Lout.kind = FENC_LAYOUT_VECTOR;
  Lout.bs = Lin.bs; Lout.c = dout; Lout.h = 1; Lout.w = 1;
  Lout.bsg = bsg; Lout.nbg = Lin.nbg; Lout.cpc = 1; Lout.ncg = 1; Lout.S = 1; Lout.m = 1; Lout.M = 1;
  Lout.d = d;
  Lout.nfeat = dout;
  Lout.pos.resize(dout);
  for (int i = 0; i < dout; i++) Lout.pos[i] = i;
  Lout.level = lvl - 1;
  Lout.scale = C.Delta;
  if (shape_only) return nullptr;
  int e = 0;
  while ((1 << e) < d) e++;
  const int n1 = 1 << ((e + 1) / 2), n2 = d / n1;
  std::vector<double> Wp((size_t)d * d, 0.0);
  std::vector<char> colused(d, 0);
  for (int f = 0; f < din; f++) colused[Lin.pos[f]] = 1;
  for (int i = 0; i < dout; i++)
    for (int f = 0; f < din; f++) Wp[(size_t)i * d + Lin.pos[f]] = W[(size_t)i * din + f];
  auto diag_active = [&](int kd) {
    for (int i = 0; i < dout; i++)
      if (colused[(i + kd) % d]) return true;
    return false;
  };
  auto P = new FcPlan;
  P->out = Lout;
  P->level = lvl;
  P->n_in = Lin.n_ct();
  P->n_out = Lout.n_ct();
  std::vector<char> baby(n1, 0), giant(n2, 0);
  for (int g = 0; g < n2; g++)
    for (int b = 0; b < n1; b++)
      if (diag_active(g * n1 + b)) baby[b] = giant[g] = 1;
  const double dp = ((double)C.primes[lvl] * C.Delta) / Lin.scale;
  std::vector<std::vector<double>> slots;
  std::vector<int> pid((size_t)n1 * n2, -1);
  for (int g = 0; g < n2; g++)
    for (int b = 0; b < n1; b++) {
      const int kd = g * n1 + b;
      if (!diag_active(kd)) continue;
      std::vector<double> z(C.ns);
      for (int l = 0; l < C.ns; l++) {
        const int i = posmod((long long)l - (long long)g * n1 * bsg, C.ns) / bsg;
        z[l] = Wp[(size_t)i * d + (i + kd) % d];
      }
      pid[(size_t)g * n1 + b] = (int)slots.size();
      slots.push_back(std::move(z));
    }
  const u64* pts = encode_plaintexts(C, slots, dp, lvl, P->owned);
  const long long pe = (long long)(lvl + 1) * C.N;
  std::vector<std::pair<int, long long>> copies;
  std::vector<int> bidx(n1, -1);
  int nb = 0;
  for (int b = 1; b < n1; b++)
    if (baby[b]) bidx[b] = nb++;
  for (int t = 0; t < P->n_in; t++)
    for (int b = 1; b < n1; b++)
      if (baby[b]) copies.push_back({t, (long long)b * bsg});
  P->rot = make_rot_stage(C, copies, P->owned);
  GmacBuild b0, br;
  std::vector<int> so, sb;
  std::vector<std::vector<std::pair<int, long long>>> st;
  for (int t = 0; t < P->n_in; t++) {
    auto in_id = [&](int b) { return b == 0 ? t : P->n_in + t * nb + bidx[b]; };
    std::vector<std::pair<int, long long>> tl;
    for (int g = 0; g < n2; g++) {
      if (g > 0 && !giant[g]) continue;
      GmacBuild& gb = g == 0 ? b0 : br;
      for (int b = 0; b < n1; b++) {
        const int id = pid[(size_t)g * n1 + b];
        if (id < 0) continue;
        gb.add_group(pts + id * pe);
        gb.add_term(in_id(b), -1);
        gb.end_group();
      }
      gb.end_output();
      if (g > 0) tl.push_back({P->n_zr++, (long long)g * n1 * bsg});
    }
    if (!tl.empty()) {
      so.push_back(t);
      sb.push_back(t);
      st.push_back(tl);
    }
  }
  P->g0 = make_gmac(C, b0, {}, lvl, P->owned);
  P->gr = make_gmac(C, br, {}, lvl, P->owned);
  P->sum = make_sum_stage(C, so, sb, st, P->owned, P->n_zr);
  if (bias) {
    P->has_bias = true;
    P->bias = make_bias(C, Lout, bias, P->owned);
  }
  return P;
}

static void run_fc(Ctx& C, const FcPlan& P, const u64* in, u64* out, fb::Stream s) {
  const int lvl = P.level, nl = lvl + 1;
  const long long ce = ct_elems(C, lvl), ps = (long long)nl * C.N;
  Scope sc(C.arena);
  u64* copies = (u64*)C.arena.get((size_t)std::max(1, P.rot.n) * ce * 8, s);
  u64* y = (u64*)C.arena.get((size_t)P.n_out * ce * 8, s);
  u64* zr = (u64*)C.arena.get((size_t)std::max(1, P.n_zr) * ce * 8, s);
  run_rot_stage(C, lvl, P.rot, in, copies, s);
  run_gmac(C, nl, P.g0, in, ce, ps, P.n_in, copies, ce, ps, y, ce, ps, s);
  run_gmac(C, nl, P.gr, in, ce, ps, P.n_in, copies, ce, ps, zr, ce, ps, s);
  run_sum_stage(C, lvl, P.sum, zr, y, y, s);
  if (P.has_bias) {
    u64* t = (u64*)C.arena.get((size_t)P.n_out * ct_elems(C, lvl - 1) * 8, s);
    rescale(C, lvl, y, P.n_out, t, s);
    run_bias(C, P.bias, lvl - 1, t, out, P.n_out, s);
  } else {
    rescale(C, lvl, y, P.n_out, out, s);
  }
  C.cnt.rot_other += P.rot.n + P.n_zr;
  C.cnt.keyswitch += P.rot.n + P.n_zr;
  C.cnt.pmult += P.g0.n_masked + P.gr.n_masked;
  C.cnt.cts_out += P.n_out;
}

// ---------------------------------------------------------------- batch-group tiles
// Batch groups share no ciphertext, so an operation on cnt of them is the
// same operation on a smaller batch: its plan is the one of that batch.
static Layout sub_layout(const Layout& L, int cnt) {
  Layout T = L;
  T.nbg = cnt;
  T.bs = cnt * L.bsg;
  return T;
}
static int cts_per_group(const Layout& L) { return L.kind == FENC_LAYOUT_FRAGMENT ? L.ncg * L.S * L.S : 1; }

// batch groups per tile for `per_group` bytes of workspace per group
static int tile_groups(const Ctx& C, int nbg, double per_group) {
  if (nbg <= 1 || C.ws_limit <= 0 || per_group * nbg <= (double)C.ws_limit) return nbg;
  return std::max(1, std::min(nbg, (int)((double)C.ws_limit / per_group)));
}

// workspace of one run of a key-switch-free or key-switching linear layer:
// outputs and outer diagonals, rotated copies, the larger ModUp output
static double conv_ws_bytes(const Ctx& C, int level, bool pq, int n_src, int n_copies, int n_in, int n_out, int n_zr) {
  const int nl = level + 1, le = nl + C.K, beta = (nl + C.alpha - 1) / C.alpha;
  const double w = (double)C.N * 8, ce = 2.0 * nl * w, ee = 2.0 * le * w, ext = (double)beta * le * w;
  double b = (n_out + n_zr) * ce + n_out * ce;   // y and z_r, and the rescale's lift
  if (pq) b += (n_copies + n_in) * ee + (n_out + n_zr) * ee;
  else b += std::max(1, n_copies) * ce;
  return b + std::max((double)n_src, (double)n_zr) * ext;
}

// ---------------------------------------------------------------- plan cache
// Modelled HBM traffic, in units of N words, of what the two hoisting
// schedules do differently in a layer with n_rot hoisted rotations.
// Schedule 0 moves every rotated copy down (inverse NTT of the 2K special
// limbs, base conversion, NTT of 2 nl limbs with the tail: about 10K + 14 nl)
// and combines over the nl limbs of Q_l.  Schedule 1 keeps the copies in
// Q_l U P, lifts the n_lift unrotated inputs, combines over nl + K limbs and
// moves the n_md combined ciphertexts down.  mac_words: words per
// (coefficient, limb) the combination moves.  Everything the schedules share
// (ModUp, key reads, outer rotations, rescale) is left out.
static double hoist_traffic(const Ctx& C, int level, bool pq, int n_rot, int n_md, int n_lift, double mac_words) {
  const double nl = level + 1, K = C.K, le = nl + K, md = 10 * K + 14 * nl;
  if (!pq) return n_rot * (2 * le + md) + mac_words * nl;
  return n_rot * 2 * le + n_lift * 2 * (nl + le) + mac_words * le + n_md * md;
}

static double mac_words(const GmacStage& g) {
  double w = 0;
  for (const MacSeg& sg : g.batched.seg) w += sg.words;
  return w;
}

// A hoisted layer's plan under the context's mode: 0 or 1 as set; 2 builds
// the schedule-0 plan, models both schedules on it (cost returns their
// traffic) and rebuilds under schedule 1 when that moves fewer words.  The
// schedule is kept in the plan (it changes residues).
template <class T, class B, class Cost>
static T* build_hoisted(Ctx& C, B build, Cost cost) {
  if (C.hoist != 2) return build(C.hoist == 1);
  T* p0 = build(false);
  const std::pair<double, double> c = cost(*p0);
  if (!(c.second < c.first)) return p0;
  dfree_all(C, p0->owned);
  delete p0;
  return build(true);
}

template <class T, class F>
static T& cached(Ctx& C, const std::string& key, F build) {
  auto it = C.plans.find(key);
  if (it != C.plans.end()) return *(T*)it->second.get();
  T* p = build();
  C.plans[key].reset(p);
  return *p;
}

// ================================================================ network planning
// Key switches of a convolution on input layout Lin, without building it:
// the same term enumeration as build_conv (distinct rotated copies (source
// ciphertext, shift != 0): inner rotations; outputs with a nonzero diagonal r:
// outer rotations, one per (output, r >= 1)), and its scalar MAC terms in the
// mask-basis form (one per output, tap and (channel position, diagonal) pair
// that connects an input channel to an output channel).  Shapes only.
static void conv_keyswitches(const Ctx& C, const Layout& Lin, int cout, int k, int stride, int pad, int groups,
                             long long& inner, long long& outer, long long& terms, int n1 = 1) {
  const int cin = Lin.c, S = Lin.S, m = Lin.m, bsg = Lin.bsg, cpc = Lin.cpc;
  const int gin = cin / groups, gout = cout / groups, So = S / stride, ncg_out = (cout + cpc - 1) / cpc;
  const int nd = Lin.rep ? cin : cpc, npos = ((cpc > 1) || (pad > 0)) ? cpc : 1;
  n1 = std::max(1, std::min(n1, nd));
  const int n2 = (nd + n1 - 1) / n1;
  const long long s_outer = (long long)m * m * bsg;
  auto in_channel = [&](int gi, int q) { return Lin.rep ? q % cin : gi * cpc + q; };
  auto pair_ok = [&](int ch, int o) { return ch < cin && o < cout && ch / gin == o / gout; };
  std::set<std::pair<int, long long>> copies;
  inner = outer = terms = 0;
  for (int bg = 0; bg < Lin.nbg; bg++)
    for (int go = 0; go < ncg_out; go++) {
      std::vector<char> act(n2, 0);   // giant steps with a term, the same for every (uo, vo)
      std::vector<int> gis;
      std::vector<std::vector<int>> babies;   // per active input group: the baby steps it feeds
      long long pairs = 0;                    // (q, r) pairs of the active input groups
      for (int gi = 0; gi < Lin.ncg; gi++) {
        std::vector<char> used(n1, 0);
        for (int q = 0; q < npos; q++)
          for (int r = 0; r < nd; r++)
            if (pair_ok(in_channel(gi, q), go * cpc + posmod(q - r, cpc))) {
              act[r / n1] = 1;
              used[r % n1] = 1;
              pairs++;
            }
        std::vector<int> b;
        for (int i = 0; i < n1; i++)
          if (used[i]) b.push_back(i);
        if (!b.empty()) {
          gis.push_back(gi);
          babies.push_back(b);
        }
      }
      for (int uo = 0; uo < So; uo++)
        for (int vo = 0; vo < So; vo++) {
          terms += pairs * k * k;
          if (!gis.empty())
            for (int j = 1; j < n2; j++) outer += act[j];
          for (size_t g = 0; g < gis.size(); g++)
            for (int di = 0; di < k; di++)
              for (int dj = 0; dj < k; dj++) {
                const int a = uo * stride + di - pad, b = vo * stride + dj - pad;
                const int u = posmod(a, S), dbi = floordiv(a, S), v = posmod(b, S), dbj = floordiv(b, S);
                const long long shift = posmod(((long long)dbi * m + dbj) * bsg, C.ns);
                for (int i : babies[g]) {
                  const long long sh = posmod(shift + (long long)i * s_outer, C.ns);
                  if (sh) copies.insert({((bg * Lin.ncg + gis[g]) * S + u) * S + v, sh});
                }
              }
        }
    }
  inner = (long long)copies.size();
}

// The baby step of a convolution's outer rotations under the context's
// setting: a fixed one, or (setting 0) the power of two up to C' with the
// fewest key switches (ties: the smaller).
static int conv_baby(const Ctx& C, const Layout& Lin, int cout, int k, int stride, int pad, int groups) {
  const int nd = Lin.rep ? Lin.c : Lin.cpc;
  if (C.baby > 0) return std::min(C.baby, nd);
  int best = 1;
  long long best_ks = -1;
  for (int n1 = 1; n1 <= nd; n1 *= 2) {
    long long a = 0, b = 0, t = 0;
    conv_keyswitches(C, Lin, cout, k, stride, pad, groups, a, b, t, n1);
    if (best_ks < 0 || a + b < best_ks) {
      best_ks = a + b;
      best = n1;
    }
  }
  return best;
}

// Key switches of a rot-mask-add repack from Ls to Ld: one hoisted rotation
// per distinct (source ciphertext, shift != 0) among the moves (the pairs
// repack_moves groups by).  When both layouts put the same images in a batch
// group, every image of a group gives its group's pairs, so the first image
// of each group is enough.
static long long repack_keyswitches(const Ctx& C, const Layout& Ls, const Layout& Ld) {
  if (Ls.bs != Ld.bs || Ls.c != Ld.c || Ls.h != Ld.h || Ls.w != Ld.w) fail(FENC_ELAYOUT, "repack between different tensors");
  const int step = (Ls.kind == Ld.kind || Ld.kind == FENC_LAYOUT_VECTOR) && Ls.bsg == Ld.bsg ? Ls.bsg : 1;
  std::unordered_set<unsigned long long> seen;
  std::vector<std::pair<int, int>> a, b;
  for (int n = 0; n < Ls.bs; n += step)
    for (int ch = 0; ch < Ls.c; ch++)
      for (int y = 0; y < Ls.h; y++)
        for (int x = 0; x < Ls.w; x++) {
          layout_slots(Ls, n, ch, y, x, a);
          layout_slots(Ld, n, ch, y, x, b);
          for (auto& d : b) {
            const long long delta = posmod((long long)a[0].second - d.second, C.ns);
            if (delta) seen.insert((unsigned long long)a[0].first * (unsigned long long)C.ns + (unsigned long long)delta);
          }
        }
  return (long long)seen.size();
}

// Block sizes of every layer of a chain, chosen by dynamic programming over
// the layout after each layer: the input may be encoded at any admissible S;
// before a convolution the tensor may be repacked (rot-mask-add into a
// fragment layout of another block size, one level each, at most max_repacks)
// so that each convolution runs at the block size that is cheapest for the
// whole chain (the paper adapts S between layers with HEAR-style rot-mask-add,
// Evaluation Methodology).  Cost: key switches of convolutions, repacks,
// S = 1 poolings (three rotations per ciphertext; S >= 2 pools sum fragments)
// and the final compression into the FC vector layout.
constexpr long long kRepackElems = 1LL << 22;
// a scalar MAC term moves at most about one ciphertext of HBM traffic, a key
// switch (ModUp, key inner product, ModDown) about 10-20
constexpr double kTermsPerKeyswitch = 16.0;

struct NetPlan {
  std::vector<int> S;   // per layer: the block size it runs at
  long long ks = 0;     // key switches: rotations, repacks, relinearisations
  long long terms = 0;  // scalar MAC terms of the convolutions
  int repacks = 0;
  double cost() const { return (double)ks + (double)terms / kTermsPerKeyswitch; }
};

static NetPlan plan_network(const Ctx& C, int bs, int c, int h, int w, const fenc_layer* layers, int n,
                            int max_repacks) {
  struct St {
    Layout L;
    NetPlan p;
  };
  auto admissible = [&](const Layout& L) {
    std::vector<int> out;
    const int M = next_pow2(std::max(L.h, L.w));
    for (int S = 1; S <= M; S <<= 1)
      if ((long long)(M / S) * (M / S) <= C.ns) out.push_back(S);
    return out;
  };
  auto better = [](const NetPlan& a, const NetPlan& b) {
    if (a.cost() != b.cost()) return a.cost() < b.cost();
    return a.repacks != b.repacks ? a.repacks < b.repacks : a.S < b.S;
  };
  auto key = [](const Layout& L, int reps) {
    return std::make_tuple(L.S, L.M, L.dil, L.c, L.h, reps);
  };
  std::vector<St> cur;
  {
    Layout L0;
    L0.h = h;
    L0.w = w;
    for (int S : admissible(L0)) cur.push_back({make_fragment(C.ns, C.L, C.Delta, bs, c, h, w, S), NetPlan{}});
  }
  for (int li = 0; li < n; li++) {
    const fenc_layer& ly = layers[li];
    std::map<decltype(key(Layout(), 0)), St> next;
    auto offer = [&](St s) {
      auto kk = key(s.L, s.p.repacks);
      auto it = next.find(kk);
      if (it == next.end() || better(s.p, it->second.p)) next[kk] = std::move(s);
    };
    for (const St& st : cur) {
      switch (ly.kind) {
        case FENC_LAYER_CONV: {
          std::vector<std::pair<Layout, long long>> starts;   // (layout the conv runs on, repack cost)
          if (st.L.dil == 1) starts.push_back({st.L, 0});
          // repacks are offered for tensors up to kRepackElems elements (their
          // count walks every element)
          const bool small = (long long)bs * st.L.c * st.L.h * st.L.w <= kRepackElems;
          if (li > 0 && st.p.repacks < max_repacks && small)
            for (int S2 : admissible(st.L)) {
              if (S2 == st.L.S && st.L.dil == 1) continue;
              Layout R = make_fragment(C.ns, st.L.level, st.L.scale, bs, st.L.c, st.L.h, st.L.w, S2);
              starts.push_back({R, repack_keyswitches(C, st.L, R)});
            }
          for (auto& sv : starts) {
            const Layout& Lc = sv.first;
            if (ly.stride < 1 || Lc.S % ly.stride || ly.groups < 1 || Lc.c % ly.groups || ly.cout % ly.groups)
              continue;
            Layout Lo;
            try {
              build_conv(*(Ctx*)&C, Lc, nullptr, ly.cout, ly.k, ly.stride, ly.pad, ly.groups, 0, nullptr, true, Lo);
            } catch (const Error&) {
              continue;
            }
            long long in = 0, out = 0, tm = 0;
            conv_keyswitches(C, Lc, ly.cout, ly.k, ly.stride, ly.pad, ly.groups, in, out, tm,
                             conv_baby(C, Lc, ly.cout, ly.k, ly.stride, ly.pad, ly.groups));
            St ns{Lo, st.p};
            ns.p.S.push_back(Lc.S);
            ns.p.ks += sv.second + in + out;
            ns.p.terms += tm;
            ns.p.repacks += sv.second > 0 || Lc.S != st.L.S || Lc.dil != st.L.dil;
            offer(std::move(ns));
          }
          break;
        }
        case FENC_LAYER_POOL: {
          Layout Lo;
          try {
            build_pool(*(Ctx*)&C, st.L, true, Lo);
          } catch (const Error&) {
            break;
          }
          St ns{Lo, st.p};
          ns.p.S.push_back(st.L.S);
          if (st.L.S == 1) ns.p.ks += 3LL * st.L.n_ct();
          offer(std::move(ns));
          break;
        }
        case FENC_LAYER_ACT: {   // relinearisations: one per ciphertext, two for degree 3
          St ns = st;
          ns.p.S.push_back(st.L.S);
          ns.p.ks += (long long)st.L.n_ct() * (ly.k >= 3 ? 2 : 1);
          offer(std::move(ns));
          break;
        }
        case FENC_LAYER_COMPRESS: {
          St ns = st;
          ns.p.S.push_back(st.L.S);
          ns.p.ks += repack_keyswitches(C, st.L, vector_target(C, st.L));
          offer(std::move(ns));
          break;
        }
        default:
          fail(FENC_EINVAL, "unknown layer kind");
      }
    }
    cur.clear();
    for (auto& kv : next) cur.push_back(std::move(kv.second));
    if (cur.empty()) fail(FENC_EUNSUPPORTED, "no block size admits layer " + std::to_string(li));
  }
  const St* best = &cur[0];
  for (const St& s : cur)
    if (better(s.p, best->p)) best = &s;
  return best->p;
}

// ================================================================ C ABI
#define API_BEGIN try {
#define API_END                                                  \
  }                                                              \
  catch (const fr::Error& e) {                                   \
    g_err = e.what();                                            \
    return e.code;                                               \
  }                                                              \
  catch (const std::exception& e) {                              \
    g_err = e.what();                                            \
    return strstr(e.what(), "out of memory") ? FENC_ENOMEM : FENC_EHIP; \
  }                                                              \
  return FENC_OK;

extern "C" {

const char* fenc_last_error(void) { return g_err.c_str(); }

static int ctx_create(const fenc_params* p, fenc_ctx** out, bool with_sk);

int fenc_ctx_create(const fenc_params* p, fenc_ctx** out) { return ctx_create(p, out, true); }
int fenc_ctx_create_server(const fenc_params* p, fenc_ctx** out) { return ctx_create(p, out, false); }

static int ctx_create(const fenc_params* p, fenc_ctx** out, bool with_sk) {
  API_BEGIN
  if (!p || !out) fail(FENC_EINVAL, "null argument");
  *out = nullptr;
  if (p->log_n < 3 || p->log_n > 17) fail(FENC_EINVAL, "log_n must be in [3, 17]");
  if (p->n_q < 2 || p->n_p < 1 || p->dnum < 1 || p->dnum > p->n_q) fail(FENC_EINVAL, "bad prime counts");
  if (p->q_bits > 50 || p->q_bits < 20 || p->p_bits != p->q_bits) fail(FENC_EINVAL, "primes must share one bit size <= 50");
  const int alpha = (p->n_q + p->dnum - 1) / p->dnum;
  if ((int)p->n_p < alpha) fail(FENC_EINVAL, "need at least one special prime per digit limb");
  if (alpha > 16 || p->n_p > 16) fail(FENC_EUNSUPPORTED, "digit or special-prime count above 16");
  if (p->n_q + p->n_p > 100) fail(FENC_EUNSUPPORTED, "too many primes");
  if (p->log2_scale < 1 || p->log2_scale >= p->q_bits) fail(FENC_EINVAL, "scale must be below the primes");
  std::unique_ptr<fenc_ctx> C(new fenc_ctx);
  C->prm = *p;
  C->logn = p->log_n;
  C->N = 1 << p->log_n;
  C->ns = C->N / 2;
  C->L = p->n_q - 1;
  C->K = p->n_p;
  C->alpha = alpha;
  C->ndig = (p->n_q + alpha - 1) / alpha;
  C->np = p->n_q + p->n_p;
  C->Delta = std::ldexp(1.0, (int)p->log2_scale);
  C->primes = fh::ntt_primes(p->q_bits, p->log_n, p->n_q, {});
  auto ps = fh::ntt_primes(p->p_bits, p->log_n, p->n_p, C->primes);
  C->primes.insert(C->primes.end(), ps.begin(), ps.end());
  for (uint64_t q : C->primes) C->psi.push_back(fh::root_2n(q, p->log_n));
  C->has_sk = with_sk;
  if (with_sk) {
    C->s.resize(C->N);
    for (int i = 0; i < C->N; i++) C->s[i] = fh::draw_ternary(p->seed, fh::tag::secret, i);
  }
  *out = C.release();
  API_END
}

void fenc_ctx_destroy(fenc_ctx* ctx) {
  try {
    delete ctx;
  } catch (...) {
  }
}

int fenc_ctx_primes(const fenc_ctx* ctx, uint64_t* out) {
  API_BEGIN
  if (!ctx || !out) fail(FENC_EINVAL, "null argument");
  for (size_t i = 0; i < ctx->primes.size(); i++) out[i] = ctx->primes[i];
  API_END
}

int fenc_set_mode(fenc_ctx* ctx, int mode) {
  API_BEGIN
  if (!ctx || (mode != FENC_MODE_BATCHED && mode != FENC_MODE_PER_OP)) fail(FENC_EINVAL, "bad mode");
  ctx->mode = mode;
  API_END
}

int fenc_set_plaintext_budget(fenc_ctx* ctx, int64_t bytes) {
  API_BEGIN
  if (!ctx || bytes < 0) fail(FENC_EINVAL, "bad budget");
  ctx->pt_budget = bytes;
  API_END
}

int fenc_set_own_copy_limit(fenc_ctx* ctx, int64_t bytes) {
  API_BEGIN
  if (!ctx || bytes < 0) fail(FENC_EINVAL, "bad own-limb copy limit");
  ctx->own_copy = bytes;
  API_END
}

int fenc_set_workspace_limit(fenc_ctx* ctx, int64_t bytes) {
  API_BEGIN
  if (!ctx || bytes < 0) fail(FENC_EINVAL, "bad workspace limit");
  ctx->ws_limit = bytes;
  API_END
}

int fenc_profile_kernel(fenc_ctx* ctx, const char* name) {
  API_BEGIN
  if (!ctx) fail(FENC_EINVAL, "null argument");
  for (auto& r : ctx->prof) {
    fb::event_destroy(r.a);
    fb::event_destroy(r.b);
  }
  ctx->prof.clear();
  ctx->prof_kernel = name ? name : "";
  API_END
}

int fenc_profile_result(fenc_ctx* ctx, double* total_ms, int64_t* launches, double* bytes) {
  API_BEGIN
  if (!ctx || !total_ms || !launches || !bytes) fail(FENC_EINVAL, "null argument");
  double ms = 0, b = 0;
  for (auto& r : ctx->prof) {
    ms += fb::event_elapsed_ms(r.a, r.b);
    b += r.bytes;
  }
  *total_ms = ms;
  *launches = (int64_t)ctx->prof.size();
  *bytes = b;
  API_END
}

int fenc_profile_summary(fenc_ctx* ctx, char* buf, int64_t len) {
  API_BEGIN
  if (!ctx || !buf || len < 1) fail(FENC_EINVAL, "null argument");
  std::map<std::string, std::tuple<double, int64_t, double, double>> agg;
  for (auto& r : ctx->prof) {
    auto& e = agg[r.name];
    std::get<0>(e) += fb::event_elapsed_ms(r.a, r.b);
    std::get<1>(e) += 1;
    std::get<2>(e) += r.bytes;
    std::get<3>(e) += r.ops;
  }
  std::ostringstream o;
  o.precision(17);
  for (auto& kv : agg)
    o << kv.first << ' ' << std::get<0>(kv.second) << ' ' << std::get<1>(kv.second) << ' ' << std::get<2>(kv.second)
      << ' ' << std::get<3>(kv.second) << '\n';
  const std::string t = o.str();
  if ((int64_t)t.size() + 1 > len) fail(FENC_EINVAL, "summary buffer too small");
  std::memcpy(buf, t.c_str(), t.size() + 1);
  API_END
}

int fenc_stats(const fenc_ctx* ctx, fenc_counters* out) {
  API_BEGIN
  if (!ctx || !out) fail(FENC_EINVAL, "null argument");
  *out = ctx->cnt;
  API_END
}

void fenc_stats_reset(fenc_ctx* ctx) {
  if (ctx) ctx->cnt = fenc_counters{};
}

int64_t fenc_device_bytes(const fenc_ctx* ctx) { return ctx ? ctx->dev_bytes + (int64_t)ctx->arena.bytes() : 0; }

int fenc_keygen(fenc_ctx* ctx, const int32_t* rot_steps, uint32_t n_steps, int relin, int strict) {
  API_BEGIN
  if (!ctx || (n_steps && !rot_steps)) fail(FENC_EINVAL, "null argument");
  ctx->strict = false;
  ensure_device(*ctx);
  for (uint32_t i = 0; i < n_steps; i++) {
    const uint64_t g = galois(*ctx, rot_steps[i]);
    if (g != 1) get_key(*ctx, g);
  }
  if (relin) get_key(*ctx, 0);
  ctx->strict = strict != 0;
  API_END
}

int fenc_key_export(fenc_ctx* ctx, int32_t shift, uint64_t* out) {
  API_BEGIN
  if (!ctx || !out) fail(FENC_EINVAL, "null argument");
  ensure_device(*ctx);
  const uint64_t g = shift == INT32_MIN ? 0 : galois(*ctx, shift);
  const uint64_t* key = get_key(*ctx, g);
  const int np = ctx->np, nd = ctx->ndig, N = ctx->N;
  std::vector<void*> tmp;
  uint64_t* t = (uint64_t*)dalloc(*ctx, (size_t)nd * 2 * np * N * 8, tmp);
  ntt(*ctx, true, key, t, (long long)np * N, (long long)np * N, nd * 2 * np, np, identity_map(np), nullptr);
  fb::sync(nullptr);
  fb::d2h(out, t, (size_t)nd * 2 * np * N * 8);
  dfree_all(*ctx, tmp);
  API_END
}

int fenc_key_list(const fenc_ctx* ctx, uint64_t* galois, int32_t cap) {
  if (!ctx || cap < 0 || (cap > 0 && !galois)) {
    g_err = "bad argument";
    return FENC_EINVAL;
  }
  int n = 0;
  for (auto& kv : ctx->keys) {
    if (n < cap) galois[n] = kv.first;
    n++;
  }
  return n;
}

static void check_galois(const Ctx& C, uint64_t g) {
  if (g != 0 && (g % 2 == 0 || g >= 2ull * C.N || g == 1)) fail(FENC_EINVAL, "not a Galois element of a rotation");
}

int fenc_key_export_galois(fenc_ctx* ctx, uint64_t g, uint64_t* out) {
  API_BEGIN
  if (!ctx || !out) fail(FENC_EINVAL, "null argument");
  check_galois(*ctx, g);
  ensure_device(*ctx);
  const uint64_t* key = get_key(*ctx, g);
  const int np = ctx->np, nd = ctx->ndig, N = ctx->N;
  std::vector<void*> tmp;
  uint64_t* t = (uint64_t*)dalloc(*ctx, (size_t)nd * 2 * np * N * 8, tmp);
  ntt(*ctx, true, key, t, (long long)np * N, (long long)np * N, nd * 2 * np, np, identity_map(np), nullptr);
  fb::sync(nullptr);
  fb::d2h(out, t, (size_t)nd * 2 * np * N * 8);
  dfree_all(*ctx, tmp);
  API_END
}

int fenc_key_import(fenc_ctx* ctx, uint64_t g, const uint64_t* in) {
  API_BEGIN
  if (!ctx || !in) fail(FENC_EINVAL, "null argument");
  fenc_ctx& C = *ctx;
  check_galois(C, g);
  if (C.keys.count(g)) fail(FENC_EINVAL, "the context already holds this key");
  ensure_device(C);
  const int np = C.np, nd = C.ndig, N = C.N;
  for (size_t i = 0; i < (size_t)nd * 2 * np * N; i++)
    if (in[i] >= C.primes[(i / N) % np]) fail(FENC_EINVAL, "key residue out of range");
  std::vector<uint64_t> h(in, in + (size_t)nd * 2 * np * N);
  uint64_t* key = upload(C, h, C.owned);
  ntt(C, false, key, key, (long long)np * N, (long long)np * N, nd * 2 * np, np, identity_map(np), nullptr);
  fb::sync(nullptr);
  C.keys[g] = key;
  API_END
}

int fenc_plan_layout(const fenc_ctx* ctx, uint32_t bs, uint32_t c, uint32_t h, uint32_t w, uint32_t k_next,
                     uint32_t cout_next, int32_t s_override, fenc_layout* out) {
  API_BEGIN
  if (!ctx || !out) fail(FENC_EINVAL, "null argument");
  Layout L = plan_fragment(ctx->ns, ctx->L, ctx->Delta, bs, c, h, w, k_next, cout_next, s_override);
  *out = to_pub(*(fenc_ctx*)ctx, L);
  API_END
}

int fenc_plan_network(const fenc_ctx* ctx, uint32_t bs, uint32_t c, uint32_t h, uint32_t w, const fenc_layer* layers,
                      uint32_t n_layers, int32_t max_repacks, int32_t* block_size, int64_t* keyswitches,
                      int64_t* mac_terms) {
  API_BEGIN
  if (!ctx || !layers || !block_size || n_layers < 1 || max_repacks < 0) fail(FENC_EINVAL, "bad argument");
  const NetPlan p = plan_network(*ctx, (int)bs, (int)c, (int)h, (int)w, layers, (int)n_layers, max_repacks);
  for (uint32_t i = 0; i < n_layers; i++) block_size[i] = p.S[i];
  if (keyswitches) *keyswitches = p.ks;
  if (mac_terms) *mac_terms = p.terms;
  API_END
}

int fenc_conv2d_keyswitches(const fenc_ctx* ctx, const fenc_layout* in, uint32_t cout, uint32_t k, uint32_t stride,
                            uint32_t pad, uint32_t groups, int64_t* inner, int64_t* outer, int64_t* mac_terms) {
  API_BEGIN
  if (!ctx || !in || !inner || !outer) fail(FENC_EINVAL, "null argument");
  Layout Lin = from_pub(*ctx, in), Lo;
  build_conv(*(Ctx*)ctx, Lin, nullptr, cout, k, stride, pad, groups, 0, nullptr, true, Lo);   // shape checks
  long long a = 0, b = 0, t = 0;
  conv_keyswitches(*ctx, Lin, cout, k, stride, pad, groups, a, b, t, conv_baby(*ctx, Lin, cout, k, stride, pad, groups));
  *inner = a;
  *outer = b;
  if (mac_terms) *mac_terms = t;
  API_END
}

int fenc_compress_keyswitches(const fenc_ctx* ctx, const fenc_layout* in, const fenc_layout* target, int64_t* ks) {
  API_BEGIN
  if (!ctx || !in || !ks) fail(FENC_EINVAL, "null argument");
  const Layout Lin = from_pub(*ctx, in);
  Layout Lt;
  if (target) {
    Lt = from_pub(*ctx, target);
    Lt.level = Lin.level;
  }
  Layout Lout;
  build_compress(*(Ctx*)ctx, Lin, target ? &Lt : nullptr, true, Lout);   // the layout compress would produce
  *ks = repack_keyswitches(*ctx, Lin, Lout);
  API_END
}

int fenc_plan_tokens(const fenc_ctx* ctx, uint32_t n, uint32_t E, uint32_t S, uint32_t group, fenc_layout* out) {
  API_BEGIN
  if (!ctx || !out) fail(FENC_EINVAL, "null argument");
  *out = to_pub(*(fenc_ctx*)ctx, make_tokens(ctx->ns, ctx->L, ctx->Delta, (int)n, (int)E, (int)S, (int)group));
  API_END
}

int fenc_layout_n_ct(const fenc_layout* lay) {
  if (!lay) return FENC_EINVAL;
  if (lay->kind == FENC_LAYOUT_TOKENS) return lay->n_bg * lay->S * lay->n_cg;
  return lay->kind == FENC_LAYOUT_FRAGMENT ? lay->n_bg * lay->n_cg * lay->S * lay->S : lay->n_bg;
}

int64_t fenc_ct_bytes(const fenc_ctx* ctx, const fenc_layout* lay) {
  if (!ctx || !lay) return FENC_EINVAL;
  return (int64_t)fenc_layout_n_ct(lay) * 2 * (lay->level + 1) * ctx->N * 8;
}

int fenc_layout_slot(const fenc_ctx* ctx, const fenc_layout* lay, int b, int ch, int y, int x, int32_t* ct,
                     int32_t* slot) {
  API_BEGIN
  if (!ctx || !ct || !slot) fail(FENC_EINVAL, "null argument");
  Layout L = from_pub(*ctx, lay);
  if (b < 0 || b >= L.bs || ch < 0 || ch >= L.c || y < 0 || y >= L.h || x < 0 || x >= L.w) fail(FENC_EINVAL, "element out of range");
  std::vector<std::pair<int, int>> sl;
  layout_slots(L, b, ch, y, x, sl);
  *ct = sl[0].first;
  *slot = sl[0].second;
  API_END
}

int fenc_layout_map(const fenc_ctx* ctx, const fenc_layout* lay, int32_t* pos) {
  API_BEGIN
  if (!ctx || !pos) fail(FENC_EINVAL, "null argument");
  Layout L = from_pub(*ctx, lay);
  if (L.kind != FENC_LAYOUT_VECTOR) fail(FENC_ELAYOUT, "not a vector layout");
  for (int i = 0; i < L.nfeat; i++) pos[i] = L.pos[i];
  API_END
}

int fenc_encode_int(int32_t log_n, const double* z, double scale, int64_t* m) {
  API_BEGIN
  if (!z || !m || log_n < 2 || log_n > 17) fail(FENC_EINVAL, "bad argument");
  fh::encode_real(log_n, z, scale, m);
  API_END
}

uint64_t fenc_sample_word(uint64_t seed, uint64_t tag, uint64_t i) { return fh::stream_word(seed, tag, i); }
int fenc_sample_gauss(uint64_t seed, uint64_t tag, uint64_t i) { return fh::draw_gauss(seed, tag, i); }

int fenc_encode_slots(fenc_ctx* ctx, const double* z, int32_t level, double scale, uint64_t* pt) {
  API_BEGIN
  if (!ctx || !z || !pt || level < 0 || level > ctx->L) fail(FENC_EINVAL, "bad argument");
  std::vector<int64_t> m(ctx->N);
  fh::encode_real(ctx->logn, z, scale, m.data());
  for (int i = 0; i <= level; i++) {
    const int64_t q = (int64_t)ctx->primes[i];
    for (int c = 0; c < ctx->N; c++) {
      int64_t v = m[c] % q;
      pt[(size_t)i * ctx->N + c] = (uint64_t)(v < 0 ? v + q : v);
    }
  }
  API_END
}

int fenc_encode_fragment(fenc_ctx* ctx, const double* x, const fenc_layout* lay, uint64_t* pt) {
  API_BEGIN
  if (!ctx || !x || !pt) fail(FENC_EINVAL, "null argument");
  Layout L = from_pub(*ctx, lay);
  const int n = L.n_ct(), N = ctx->N;
  std::vector<std::vector<double>> z(n, std::vector<double>(ctx->ns, 0.0));
  std::vector<std::pair<int, int>> sl;
  for (int b = 0; b < L.bs; b++)
    for (int ch = 0; ch < L.c; ch++)
      for (int y = 0; y < L.h; y++)
        for (int xx = 0; xx < L.w; xx++) {
          layout_slots(L, b, ch, y, xx, sl);
          const double v = x[(((size_t)b * L.c + ch) * L.h + y) * L.w + xx];
          for (auto& p : sl) z[p.first][p.second] = v;
        }
  const int nl = L.level + 1;
  const int nthr = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  for (int wk = 0; wk < nthr; wk++)
    th.emplace_back([&, wk] {
      std::vector<int64_t> m(N);
      for (int t = wk; t < n; t += nthr) {
        fh::encode_real(ctx->logn, z[t].data(), L.scale, m.data());
        for (int i = 0; i < nl; i++) {
          const int64_t q = (int64_t)ctx->primes[i];
          for (int c = 0; c < N; c++) {
            int64_t v = m[c] % q;
            pt[((size_t)t * nl + i) * N + c] = (uint64_t)(v < 0 ? v + q : v);
          }
        }
      }
    });
  for (auto& t : th) t.join();
  API_END
}

int fenc_encrypt(fenc_ctx* ctx, const uint64_t* pt, const fenc_layout* lay, uint64_t enc_seed, fenc_ctbatch* out,
                 void* stream) {
  API_BEGIN
  if (!ctx || !pt || !out) fail(FENC_EINVAL, "null argument");
  if (!ctx->has_sk) fail(FENC_ENOKEY, "server context holds no secret key: encryption is the client's");
  Layout L = from_pub(*ctx, lay);
  out->lay = *lay;
  if (!out->data) return FENC_OK;
  fenc_ctx& C = *ctx;
  ensure_device(C);
  const int n = L.n_ct(), nl = L.level + 1, N = C.N;
  std::vector<uint64_t> a((size_t)n * nl * N);
  std::vector<long long> e((size_t)n * N);
  const int nthr = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  for (int wk = 0; wk < nthr; wk++)
    th.emplace_back([&, wk] {
      for (int r = wk; r < n * nl; r += nthr) {
        const int t = r / nl, i = r % nl;
        for (int c = 0; c < N; c++) a[(size_t)r * N + c] = fh::draw_uniform(enc_seed, fh::tag::enc_a(t, i), c, C.primes[i]);
      }
      for (int t = wk; t < n; t += nthr)
        for (int c = 0; c < N; c++) e[(size_t)t * N + c] = fh::draw_gauss(enc_seed, fh::tag::enc_e(t), c);
    });
  for (auto& t : th) t.join();
  fb::Stream s = (fb::Stream)stream;
  fb::sync(s);
  std::vector<void*> tmp;
  uint64_t* da = upload(C, a, tmp);
  std::vector<uint64_t> ptv(pt, pt + (size_t)n * nl * N);
  uint64_t* dm = upload(C, ptv, tmp);
  long long* de = upload(C, e, tmp);
  std::vector<unsigned char> pr(nl);
  for (int i = 0; i < nl; i++) pr[i] = (unsigned char)i;
  unsigned char* dp = upload(C, pr, tmp);
  uint64_t* dE = (uint64_t*)dalloc(C, (size_t)n * nl * N * 8, tmp);
  ntt(C, false, da, da, (long long)nl * N, (long long)nl * N, n * nl, nl, identity_map(nl), nullptr);
  ntt(C, false, dm, dm, (long long)nl * N, (long long)nl * N, n * nl, nl, identity_map(nl), nullptr);
  fk::SmallArgs sa{de, dE, nl, C.logn, dp, C.pq};
  fb::small_to_rns({(unsigned)std::max(1, N / 256), (unsigned)(n * nl), 1}, std::min(256, N), nullptr, sa);
  ntt(C, false, dE, dE, (long long)nl * N, (long long)nl * N, n * nl, nl, identity_map(nl), nullptr);
  fk::EncArgs ea{da, dE, dm, C.s_ntt, out->data, nl, C.logn, C.pq};
  fb::enc_combine({(unsigned)std::max(1, N / 256), (unsigned)(n * nl), 1}, std::min(256, N), nullptr, ea);
  fb::sync(nullptr);
  dfree_all(C, tmp);
  API_END
}

static void decrypt_limbs(fenc_ctx& C, const fenc_ctbatch* in, std::vector<uint64_t>& m, int limbs, fb::Stream s) {
  if (!C.has_sk) fail(FENC_ENOKEY, "server context holds no secret key: decryption is the client's");
  Layout L = from_pub(C, &in->lay);
  ensure_device(C);
  const int n = L.n_ct(), nl = L.level + 1, N = C.N;
  fb::sync(s);
  std::vector<void*> tmp;
  uint64_t* dm = (uint64_t*)dalloc(C, (size_t)n * nl * N * 8, tmp);
  fk::DecArgs da{in->data, C.s_ntt, dm, nl, C.logn, C.pq};
  fb::dec_combine({(unsigned)std::max(1, N / 256), (unsigned)(n * nl), 1}, std::min(256, N), nullptr, da);
  fk::PrimeMap pm = identity_map(nl);
  for (int i = limbs; i < nl; i++) pm.p[i] = fk::kSkip;
  ntt(C, true, dm, dm, (long long)nl * N, (long long)nl * N, n * nl, nl, pm, nullptr);
  fb::sync(nullptr);
  m.resize((size_t)n * nl * N);
  fb::d2h(m.data(), dm, m.size() * 8);
  dfree_all(C, tmp);
}

int fenc_decrypt_raw(fenc_ctx* ctx, const fenc_ctbatch* in, uint64_t* m, void* stream) {
  API_BEGIN
  if (!ctx || !m) fail(FENC_EINVAL, "null argument");
  check_batch(*ctx, in, true);
  std::vector<uint64_t> v;
  decrypt_limbs(*ctx, in, v, in->lay.level + 1, (fb::Stream)stream);
  std::memcpy(m, v.data(), v.size() * 8);
  API_END
}

int fenc_decrypt(fenc_ctx* ctx, const fenc_ctbatch* in, double* x, void* stream) {
  API_BEGIN
  if (!ctx || !x) fail(FENC_EINVAL, "null argument");
  check_batch(*ctx, in, true);
  fenc_ctx& C = *ctx;
  Layout L = from_pub(C, &in->lay);
  std::vector<uint64_t> m;
  decrypt_limbs(C, in, m, 1, (fb::Stream)stream);
  const int n = L.n_ct(), nl = L.level + 1, N = C.N;
  const uint64_t q0 = C.primes[0];
  std::vector<std::vector<double>> z(n, std::vector<double>(C.ns));
  std::vector<int64_t> mi(N);
  for (int t = 0; t < n; t++) {
    const uint64_t* r = &m[(size_t)t * nl * N];
    for (int c = 0; c < N; c++) mi[c] = r[c] > (q0 - 1) / 2 ? (int64_t)r[c] - (int64_t)q0 : (int64_t)r[c];
    fh::decode_real(C.logn, mi.data(), L.scale, z[t].data());
  }
  std::vector<std::pair<int, int>> sl;
  for (int b = 0; b < L.bs; b++)
    for (int ch = 0; ch < L.c; ch++)
      for (int y = 0; y < L.h; y++)
        for (int xx = 0; xx < L.w; xx++) {
          layout_slots(L, b, ch, y, xx, sl);
          x[(((size_t)b * L.c + ch) * L.h + y) * L.w + xx] = z[sl[0].first][sl[0].second];
        }
  API_END
}

int fenc_ct_export(fenc_ctx* ctx, const fenc_ctbatch* in, uint64_t* host, void* stream) {
  API_BEGIN
  if (!ctx || !host) fail(FENC_EINVAL, "null argument");
  check_batch(*ctx, in, true);
  fenc_ctx& C = *ctx;
  ensure_device(C);
  Layout L = from_pub(C, &in->lay);
  const int n = L.n_ct(), nl = L.level + 1, N = C.N;
  fb::sync((fb::Stream)stream);
  std::vector<void*> tmp;
  uint64_t* t = (uint64_t*)dalloc(C, (size_t)n * 2 * nl * N * 8, tmp);
  ntt(C, true, in->data, t, (long long)nl * N, (long long)nl * N, n * 2 * nl, nl, identity_map(nl), nullptr);
  fb::sync(nullptr);
  fb::d2h(host, t, (size_t)n * 2 * nl * N * 8);
  dfree_all(C, tmp);
  API_END
}

int fenc_ct_import(fenc_ctx* ctx, const uint64_t* host, fenc_ctbatch* out, void* stream) {
  API_BEGIN
  if (!ctx || !host) fail(FENC_EINVAL, "null argument");
  check_batch(*ctx, out, true);
  fenc_ctx& C = *ctx;
  ensure_device(C);
  Layout L = from_pub(C, &out->lay);
  const int n = L.n_ct(), nl = L.level + 1, N = C.N;
  fb::sync((fb::Stream)stream);
  fb::h2d(out->data, host, (size_t)n * 2 * nl * N * 8);
  ntt(C, false, out->data, out->data, (long long)nl * N, (long long)nl * N, n * 2 * nl, nl, identity_map(nl), nullptr);
  fb::sync(nullptr);
  API_END
}

int fenc_conv2d(fenc_ctx* ctx, const fenc_ctbatch* in, const double* w, const double* bias, uint32_t cout, uint32_t k,
                uint32_t stride, uint32_t pad, uint32_t groups, int32_t s_out, fenc_ctbatch* out, void* stream) {
  API_BEGIN
  if (!ctx || !w || !out) fail(FENC_EINVAL, "null argument");
  if (s_out < 0) fail(FENC_EINVAL, "s_out must be 0 (natural layout) or a block size");
  check_batch(*ctx, in, false);
  fenc_ctx& C = *ctx;
  Layout Lin = from_pub(C, &in->lay), Lout;
  if (bias)
    for (uint32_t o = 0; o < cout; o++)
      if (!std::isfinite(bias[o])) fail(FENC_EINVAL, "non-finite bias");
  build_conv(C, Lin, w, cout, k, stride, pad, groups, s_out, bias, true, Lout);
  out->lay = to_pub(C, Lout);
  if (!out->data) return FENC_OK;
  check_batch(C, in, true);
  ensure_device(C);
  const size_t nw = (size_t)cout * (Lin.c / groups) * k * k;
  const uint64_t wh = fnv(w, nw * sizeof(double)), bh = bias ? fnv(bias, cout * sizeof(double)) : 0;
  auto plan_of = [&](int cnt) -> ConvPlan& {
    const Layout Ls = sub_layout(Lin, cnt);
    std::ostringstream key;
    key << "conv|" << layout_key(Ls) << '|' << cout << ',' << k << ',' << stride << ',' << pad << ',' << groups << ','
        << wh << ',' << bh << ',' << s_out << ',' << C.pt_budget << ',' << C.hoist << ',' << C.baby;
    return cached<ConvPlan>(C, key.str(), [&] {
      const int n1 = s_out > 0 ? 1 : conv_baby(C, Ls, cout, k, stride, pad, groups);
      return build_hoisted<ConvPlan>(
          C,
          [&](bool pq) {
            Layout lo;
            return build_conv(C, Ls, w, cout, k, stride, pad, groups, s_out, bias, false, lo, pq, n1);
          },
          [&](const ConvPlan& P) {
            const double mw = mac_words(P.g0) + mac_words(P.gr);
            return std::make_pair(hoist_traffic(C, P.level, false, P.rot.n, 0, 0, mw),
                                  hoist_traffic(C, P.level, true, P.rot.n, P.n_out + P.n_zr, P.n_in, mw));
          });
    });
  };
  // a fused repack into another batch grouping cannot be split by groups
  const bool tileable = s_out == 0 || (Lout.bsg == Lin.bsg && Lout.nbg == Lin.nbg);
  int tile = Lin.nbg;
  if (Lin.nbg > 1 && C.ws_limit > 0 && tileable) {
    const ConvPlan& P1 = plan_of(1);
    tile = tile_groups(C, Lin.nbg, conv_ws_bytes(C, P1.level, P1.pq, (int)P1.rot.src.size(), P1.rot.n, P1.n_in,
                                                 P1.n_out, P1.n_zr));
  }
  const long long in_step = (long long)cts_per_group(Lin) * ct_elems(C, Lin.level);
  const long long out_step = (long long)cts_per_group(Lout) * ct_elems(C, Lout.level);
  for (int b0 = 0; b0 < Lin.nbg; b0 += tile) {
    const ConvPlan& P = plan_of(std::min(tile, Lin.nbg - b0));
    run_conv(C, P, in->data + b0 * in_step, out->data + b0 * out_step, (fb::Stream)stream);
    C.last_hoist = P.pq;
    C.last_baby = P.n1;
  }
  API_END
}

int fenc_avgpool2(fenc_ctx* ctx, const fenc_ctbatch* in, fenc_ctbatch* out, void* stream) {
  API_BEGIN
  if (!ctx || !out) fail(FENC_EINVAL, "null argument");
  check_batch(*ctx, in, false);
  fenc_ctx& C = *ctx;
  Layout Lin = from_pub(C, &in->lay), Lout;
  build_pool(C, Lin, true, Lout);
  out->lay = to_pub(C, Lout);
  if (!out->data) return FENC_OK;
  check_batch(C, in, true);
  ensure_device(C);
  auto plan_of = [&](int cnt) -> PoolPlan& {
    const Layout Ls = sub_layout(Lin, cnt);
    return cached<PoolPlan>(C, "pool|" + layout_key(Ls) + "|h" + std::to_string(C.hoist), [&] {
      return build_hoisted<PoolPlan>(
          C,
          [&](bool pq) {
            Layout lo;
            return build_pool(C, Ls, false, lo, pq);
          },
          [&](const PoolPlan& P) {
            const double mw = mac_words(P.g);
            return std::make_pair(hoist_traffic(C, P.level, false, P.rot.n, 0, 0, mw),
                                  hoist_traffic(C, P.level, true, P.rot.n, P.n_out, P.n_in, mw));
          });
    });
  };
  int tile = Lin.nbg;
  if (Lin.nbg > 1 && C.ws_limit > 0 && Lin.S == 1) {
    const PoolPlan& P1 = plan_of(1);
    tile = tile_groups(C, Lin.nbg, conv_ws_bytes(C, P1.level, P1.pq, (int)P1.rot.src.size(), P1.rot.n, P1.n_in,
                                                 P1.n_out, 0));
  }
  const long long in_step = (long long)cts_per_group(Lin) * ct_elems(C, Lin.level);
  const long long out_step = (long long)cts_per_group(Lout) * ct_elems(C, Lout.level);
  for (int b0 = 0; b0 < Lin.nbg; b0 += tile) {
    const PoolPlan& P = plan_of(std::min(tile, Lin.nbg - b0));
    run_pool(C, P, in->data + b0 * in_step, out->data + b0 * out_step, (fb::Stream)stream);
    C.last_hoist = P.pq;
  }
  API_END
}

int fenc_poly_act(fenc_ctx* ctx, const fenc_ctbatch* in, const double* coeffs, uint32_t degree, fenc_ctbatch* out,
                  void* stream) {
  API_BEGIN
  if (!ctx || !coeffs || !out) fail(FENC_EINVAL, "null argument");
  check_batch(*ctx, in, false);
  if (degree > 3) fail(FENC_EUNSUPPORTED, "polynomial degree above 3");
  fenc_ctx& C = *ctx;
  double c[4] = {0, 0, 0, 0};
  for (uint32_t i = 0; i <= degree; i++) {
    if (!std::isfinite(coeffs[i])) fail(FENC_EINVAL, "non-finite coefficient");
    c[i] = coeffs[i];
  }
  int d = (int)degree;
  while (d > 0 && c[d] == 0.0) d--;
  Layout Lin = from_pub(C, &in->lay);
  if (Lin.level < (d == 3 ? 2 : 1)) fail(FENC_ELEVEL, "no level left for the activation");
  const double s0 = Lin.scale, ql = (double)C.primes[Lin.level];
  Layout Lout = Lin;
  double S = C.Delta * ql, kk = 0, k3 = 0, Su = 0;
  if (d == 2) {
    kk = std::round((c[2] * (C.Delta * ql)) / (s0 * s0));
    if (kk == 0) kk = c[2] > 0 ? 1 : -1;
    S = ((kk * s0) * s0) / c[2];
    Lout.level = Lin.level - 1;
    Lout.scale = S / ql;
  } else if (d == 3) {
    const double q1 = (double)C.primes[Lin.level - 1];
    kk = std::round((C.Delta * ql) / (s0 * s0));
    if (kk < 1) kk = 1;
    const double s2 = ((kk * s0) * s0) / ql;
    k3 = std::round((c[3] * q1) / s0);
    if (k3 == 0) k3 = c[3] > 0 ? 1 : -1;
    Su = (k3 * s0) / c[3];
    S = s2 * Su;
    Lout.level = Lin.level - 2;
    Lout.scale = S / q1;
  } else {
    Lout.level = Lin.level - 1;
    Lout.scale = S / ql;
  }
  if (std::fabs(kk) >= 9007199254740992.0 || std::fabs(k3) >= 9007199254740992.0)
    fail(FENC_ESCALE, "activation scale factor out of range");
  out->lay = to_pub(C, Lout);
  if (!out->data) return FENC_OK;
  check_batch(C, in, true);
  ensure_device(C);
  // workspace per ciphertext: the product, its third part, the ModUp output
  // and, for degree 3, x^2 and u one level down
  const int l = Lin.level, nl1 = l + 1, beta = (nl1 + C.alpha - 1) / C.alpha;
  // ciphertexts are independent here, so tiles are runs of ciphertexts
  const double per_ct = (double)C.N * 8 * (2.0 * nl1 + nl1 + (double)beta * (nl1 + C.K) + (d == 3 ? 4.0 * l : 0.0));
  const int n_all = Lin.n_ct();
  const int tile = tile_groups(C, n_all, per_ct);
  const long long in_step = ct_elems(C, Lin.level), out_step = ct_elems(C, Lout.level);
  for (int b0 = 0; b0 < n_all; b0 += tile) {
  const int n_tile = std::min(tile, n_all - b0);
  std::ostringstream key;
  key << "poly|" << layout_key(Lin) << '|' << n_tile << '|' << fnv(c, sizeof(c));
  PolyPlan& P = cached<PolyPlan>(C, key.str(), [&] {
    auto p = new PolyPlan;
    p->out = Lout;
    p->level = Lin.level;
    p->n = n_tile;
    p->d = d;
    p->lin = d <= 1 || c[0] != 0.0 || c[1] != 0.0;   // adding zero codes changes nothing
    const int l = Lin.level;
    auto up = [&](const std::vector<d2>& v) { return upload(C, v, p->owned); };
    if (d >= 2) {
      std::vector<std::vector<KsItem>> items;
      std::vector<fk::TailItem> tails;
      const uint64_t* rk = get_key(C, 0);
      for (int b = 0; b < p->n; b++) {
        items.push_back({KsItem{b, 1u, rk}});
        tails.push_back(fk::TailItem{b, b, 0, 0});
      }
      p->ks_a = make_ks(C, items, tails, {}, p->owned);
      if (d == 3) p->ks_b = make_ks(C, items, tails, {}, p->owned);
      p->kf = up(code_residues(C, kk, l + 1));
    }
    if (d == 3) {
      p->one = up(code_residues(C, 1.0, l));
      p->k3 = up(code_residues(C, k3, l));
      p->k2c = up(code_residues(C, c[2] * Su, l));
      p->k1 = up(code_residues(C, c[1] * S / s0, l));
      p->k0 = up(code_residues(C, c[0] * S, l));
    } else {
      p->k1 = up(code_residues(C, c[1] * S / s0, l + 1));
      p->k0 = up(code_residues(C, c[0] * S, l + 1));
    }
    return p;
  });
  run_poly(C, P, in->data + b0 * in_step, out->data + b0 * out_step, (fb::Stream)stream);
  }
  API_END
}

int fenc_compress(fenc_ctx* ctx, const fenc_ctbatch* in, const fenc_layout* target, fenc_ctbatch* out, void* stream) {
  API_BEGIN
  if (!ctx || !out) fail(FENC_EINVAL, "null argument");
  check_batch(*ctx, in, false);
  fenc_ctx& C = *ctx;
  Layout Lin = from_pub(C, &in->lay), Lout, Lt;
  if (target) {
    Lt = from_pub(C, target);
    Lt.level = Lin.level;   // the target's level and scale are outputs
  }
  build_compress(C, Lin, target ? &Lt : nullptr, true, Lout);
  out->lay = to_pub(C, Lout);
  if (!out->data) return FENC_OK;
  check_batch(C, in, true);
  ensure_device(C);
  CompressPlan& P = cached<CompressPlan>(
      C, "aac|" + layout_key(Lin) + "|" + (target ? layout_key(Lt) : "") + "|h" + std::to_string(C.hoist), [&] {
        return build_hoisted<CompressPlan>(
            C, [&](bool pq) { return build_compress(C, Lin, target ? &Lt : nullptr, false, Lout, pq); },
            [&](const CompressPlan& P) {
              const double mw = mac_words(P.g);
              return std::make_pair(hoist_traffic(C, P.level, false, P.rot.n, 0, 0, mw),
                                    hoist_traffic(C, P.level, true, P.rot.n, P.n_out, P.n_in, mw));
            });
      });
  run_compress(C, P, in->data, out->data, (fb::Stream)stream);
  C.last_hoist = P.pq;
  API_END
}

int fenc_fc(fenc_ctx* ctx, const fenc_ctbatch* in, const double* w, const double* bias, uint32_t dout,
            fenc_ctbatch* out, void* stream) {
  API_BEGIN
  if (!ctx || !w || !out) fail(FENC_EINVAL, "null argument");
  check_batch(*ctx, in, false);
  fenc_ctx& C = *ctx;
  Layout Lin = from_pub(C, &in->lay), Lout;
  if (bias)
    for (uint32_t o = 0; o < dout; o++)
      if (!std::isfinite(bias[o])) fail(FENC_EINVAL, "non-finite bias");
  build_fc(C, Lin, w, dout, bias, true, Lout);
  out->lay = to_pub(C, Lout);
  if (!out->data) return FENC_OK;
  check_batch(C, in, true);
  ensure_device(C);
  std::ostringstream key;
  key << "fc|" << layout_key(Lin) << '|' << dout << ',' << fnv(w, (size_t)dout * Lin.nfeat * sizeof(double)) << ','
      << (bias ? fnv(bias, dout * sizeof(double)) : 0);
  FcPlan& P = cached<FcPlan>(C, key.str(), [&] { return build_fc(C, Lin, w, dout, bias, false, Lout); });
  run_fc(C, P, in->data, out->data, (fb::Stream)stream);
  API_END
}

int fenc_rotate(fenc_ctx* ctx, const fenc_ctbatch* in, const int32_t* shifts, uint32_t n, fenc_ctbatch* out,
                void* stream) {
  API_BEGIN
  if (!ctx || !shifts || !out || n == 0) fail(FENC_EINVAL, "bad argument");
  check_batch(*ctx, in, true);
  fenc_ctx& C = *ctx;
  Layout L = from_pub(C, &in->lay);
  check_batch(C, out, true);
  ensure_device(C);
  const int nct = L.n_ct();
  std::ostringstream key;
  key << "rot|" << L.level << ',' << nct;
  for (uint32_t i = 0; i < n; i++) {
    if (galois(C, shifts[i]) == 1) fail(FENC_EINVAL, "zero rotation");
    key << ',' << shifts[i];
  }
  struct RotPlan : Plan {
    RotStage r;
  };
  RotPlan& P = cached<RotPlan>(C, key.str(), [&] {
    auto p = new RotPlan;
    std::vector<std::pair<int, long long>> copies;
    for (int t = 0; t < nct; t++)
      for (uint32_t i = 0; i < n; i++) copies.push_back({t, shifts[i]});
    p->r = make_rot_stage(C, copies, p->owned);
    return p;
  });
  run_rot_stage(C, L.level, P.r, in->data, out->data, (fb::Stream)stream);
  C.cnt.rot_other += P.r.n;
  C.cnt.keyswitch += P.r.n;
  API_END
}

int fenc_rotate_sum(fenc_ctx* ctx, const fenc_ctbatch* z0, const fenc_ctbatch* zs, const int32_t* shifts, uint32_t n,
                    fenc_ctbatch* out, void* stream) {
  API_BEGIN
  if (!ctx || !shifts || !out || n == 0) fail(FENC_EINVAL, "bad argument");
  check_batch(*ctx, zs, true);
  check_batch(*ctx, out, true);
  fenc_ctx& C = *ctx;
  Layout L = from_pub(C, &zs->lay);
  if (z0) check_batch(C, z0, true);
  ensure_device(C);
  std::ostringstream key;
  key << "rsum|" << L.level << ',' << (z0 ? 1 : 0);
  for (uint32_t i = 0; i < n; i++) key << ',' << shifts[i];
  struct SumPlan : Plan {
    SumStage s;
  };
  SumPlan& P = cached<SumPlan>(C, key.str(), [&] {
    auto p = new SumPlan;
    std::vector<std::pair<int, long long>> t;
    for (uint32_t i = 0; i < n; i++) t.push_back({(int)i, shifts[i]});
    p->s = make_sum_stage(C, {0}, {z0 ? 0 : -1}, {t}, p->owned, (int)n);
    return p;
  });
  run_sum_stage(C, L.level, P.s, zs->data, out->data, z0 ? z0->data : nullptr, (fb::Stream)stream);
  API_END
}

int fenc_rescale(fenc_ctx* ctx, const fenc_ctbatch* in, fenc_ctbatch* out, void* stream) {
  API_BEGIN
  if (!ctx || !out) fail(FENC_EINVAL, "null argument");
  check_batch(*ctx, in, false);
  fenc_ctx& C = *ctx;
  Layout L = from_pub(C, &in->lay);
  if (L.level < 1) fail(FENC_ELEVEL, "no level left to rescale");
  Layout Lo = L;
  Lo.level = L.level - 1;
  Lo.scale = L.scale / (double)C.primes[L.level];
  out->lay = to_pub(C, Lo);
  if (!out->data) return FENC_OK;
  check_batch(C, in, true);
  ensure_device(C);
  rescale(C, L.level, in->data, L.n_ct(), out->data, (fb::Stream)stream);
  API_END
}

int fenc_rescale_noalloc(fenc_ctx* ctx, const fenc_ctbatch* in, fenc_ctbatch* out, void* stream) {
  API_BEGIN
  if (!ctx || !out) fail(FENC_EINVAL, "null argument");
  check_batch(*ctx, in, false);
  fenc_ctx& C = *ctx;
  Layout L = from_pub(C, &in->lay);
  if (L.level < 1) fail(FENC_ELEVEL, "no level left to rescale");
  Layout Lo = L;
  Lo.level = L.level - 1;
  Lo.scale = L.scale / (double)C.primes[L.level];
  out->lay = to_pub(C, Lo);
  if (!out->data) return FENC_OK;
  check_batch(C, in, true);
  if (!C.dev) fail(FENC_EINVAL, "no device tables yet: run an operation of this context on this device first");
  if (fb::device_id() != C.device) fail(FENC_EINVAL, "the context's tables live on another device");
  if (!C.lvl.count(L.level)) fail(FENC_EINVAL, "no tables for this level yet: run fenc_rescale at this level once");
  const int n = L.n_ct();
  const size_t need = rescale_ws_bytes(C, L.level, n);
  if (need > fb::kScratchBytes)
    fail(FENC_EINVAL, "rescale workspace of " + std::to_string(need) + " bytes exceeds the static scratch of " +
                          std::to_string(fb::kScratchBytes) + " bytes: split the batch");
  u64* last = (u64*)fb::scratch_base();
  u64* lift = last + (size_t)n * 2 * C.N;
  rescale_ws(C, L.level, in->data, n, out->data, (fb::Stream)stream, last, lift);
  API_END
}

int fenc_set_hoisting(fenc_ctx* ctx, int mode) {
  API_BEGIN
  if (!ctx || mode < 0 || mode > 2) fail(FENC_EINVAL, "hoisting mode must be 0, 1 or 2");
  ctx->hoist = mode;
  API_END
}

int fenc_last_hoisting(const fenc_ctx* ctx) { return ctx ? ctx->last_hoist : -1; }

int fenc_set_baby_step(fenc_ctx* ctx, int n1) {
  API_BEGIN
  if (!ctx || n1 < 0) fail(FENC_EINVAL, "baby step must be 0 (chosen per layer) or at least 1");
  ctx->baby = n1;
  API_END
}

int fenc_last_baby_step(const fenc_ctx* ctx) { return ctx ? ctx->last_baby : -1; }

int fenc_ntt_config(fenc_ctx* ctx, int32_t* out) {
  API_BEGIN
  if (!ctx || !out) fail(FENC_EINVAL, "null argument");
  for (int k = 0; k < 4; k++) {
    out[2 * k] = ctx->ntt_cfg[k][0];
    out[2 * k + 1] = ctx->ntt_cfg[k][1];
  }
  API_END
}

int fenc_set_ntt_config(fenc_ctx* ctx, const int32_t* cfg) {
  API_BEGIN
  if (!ctx || !cfg) fail(FENC_EINVAL, "null argument");
  const int n2 = (ctx->logn + 1) / 2, n1 = ctx->logn - n2;
  for (int k = 0; k < 4; k++) {
    const int rb = cfg[2 * k], t = cfg[2 * k + 1];
    const int P = (k == 0 || k == 3) ? n1 : n2, other = (k == 0 || k == 3) ? n2 : n1;
    if (rb != 3 && rb != 4) fail(FENC_EINVAL, "NTT radix bits must be 3 or 4");
    if (t < -1 || t > other || (t >= 0 && (8LL << (P + t)) > (64 << 10))) fail(FENC_EINVAL, "NTT tile out of range");
  }
  for (int k = 0; k < 4; k++) {
    ctx->ntt_cfg[k][0] = cfg[2 * k];
    ctx->ntt_cfg[k][1] = cfg[2 * k + 1];
  }
  ctx->ntt_tuned = true;   // an explicit shape is not re-tuned
  API_END
}

int fenc_ntt_rows(fenc_ctx* ctx, uint64_t* rows, const int32_t* prime, uint32_t n, int inverse) {
  API_BEGIN
  if (!ctx || !rows || !prime || n == 0 || n > (uint32_t)fk::kMaxMap) fail(FENC_EINVAL, "bad argument");
  fenc_ctx& C = *ctx;
  ensure_device(C);
  fk::PrimeMap pm;
  pm.n = (int)n;
  for (uint32_t i = 0; i < n; i++) {
    if (prime[i] < 0 || prime[i] >= C.np) fail(FENC_EINVAL, "prime index out of range");
    pm.p[i] = (unsigned char)prime[i];
  }
  std::vector<void*> tmp;
  std::vector<uint64_t> h(rows, rows + (size_t)n * C.N);
  uint64_t* d = upload(C, h, tmp);
  ntt(C, inverse != 0, d, d, C.N, C.N, (int)n, 1, pm, nullptr);
  fb::sync(nullptr);
  fb::d2h(rows, d, (size_t)n * C.N * 8);
  dfree_all(C, tmp);
  API_END
}

}  // extern "C"
