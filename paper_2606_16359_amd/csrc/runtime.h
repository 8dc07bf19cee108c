// Host runtime of the library: context, device tables, keys, workspace arena,
// key-switching pipelines and cached operation plans.  Contains no device
// code; every kernel is reached through fenc_backend.h.
#pragma once
#include <cstdint>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/fenc.h"
#include "fenc_backend.h"
#include "host_math.h"

namespace fr {

typedef uint64_t u64;
using fk::d2;

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};
[[noreturn]] inline void fail(int code, const std::string& m) { throw Error(code, m); }

// ---------------------------------------------------------------- layout
struct Layout {
  int kind = FENC_LAYOUT_FRAGMENT;
  int bs = 0, c = 0, h = 0, w = 0, M = 0, S = 0, m = 0, bsg = 0, cpc = 0, nbg = 0, ncg = 0;
  int rep = 0, dil = 1, level = 0, d = 0, nfeat = 0;
  double scale = 1.0;
  std::vector<int> pos;   // VECTOR layouts
  int n_ct() const {
    return kind == FENC_LAYOUT_FRAGMENT ? nbg * ncg * S * S : kind == FENC_LAYOUT_TOKENS ? nbg * S * ncg : nbg;
  }
};

Layout make_fragment(int ns, int level, double scale, int bs, int c, int h, int w, int S);
Layout plan_fragment(int ns, int level, double scale, int bs, int c, int h, int w, int k, int cout, int s_override);
Layout make_tokens(int ns, int level, double scale, int n, int E, int S, int group);
// first (ct, slot) of an element, plus every replica when `all`
void layout_slots(const Layout& L, int b, int ch, int y, int x, std::vector<std::pair<int, int>>& out);

// ---------------------------------------------------------------- arena
// Chunked stack workspace.  Allocation order is deterministic, so a repeated
// operation gets the same addresses (required for graph replay).  Everything
// past the current position is free; when a request fits no chunk, the free
// chunks that are too small are returned to the device (after a device-wide
// synchronisation) before a larger one is allocated, so the capacity follows
// the largest operation instead of accumulating.  Chunks used during a stream
// capture are kept: a captured graph holds their addresses.
class Arena {
 public:
  struct Mark {
    size_t chunk, off;
  };
  ~Arena();
  void* get(size_t bytes, fb::Stream s);
  Mark mark() const { return {cur_, off_}; }
  void release(Mark m) { cur_ = m.chunk; off_ = m.off; }
  size_t bytes() const;
 private:
  struct Chunk {
    char* p;
    size_t cap;
    bool pinned;   // used during a stream capture
  };
  std::vector<Chunk> chunks_;
  size_t cur_ = 0, off_ = 0;
};

struct Scope {   // releases arena allocations of one operation
  Arena& a;
  Arena::Mark m;
  explicit Scope(Arena& ar) : a(ar), m(ar.mark()) {}
  ~Scope() { a.release(m); }
};

// ---------------------------------------------------------------- device tables of a KS stage
// One item of a key-switch stage: ext ct `ct` rotated by Galois element g.
struct KsItem {
  int ct;
  unsigned g;
  const uint64_t* key;
  int c0ct = -1;   // input ct whose sigma_g(c0), times P, is folded into the accumulator (-1: none)
  int own = -1;    // input ct holding the digits' own limbs of ext ct `ct` (-1: ct itself)
};

// Device tables of a KIP + ModDown stage.  Outputs are grouped twice: in
// batched groups (up to kKipOut outputs sharing their keys) and one output per
// group for the per-op mode.
struct KipTables {
  int n = 0;                       // groups
  fk::KipGroup* groups = nullptr;
  fk::KipKey* keys = nullptr;
  int* items = nullptr;
  int* c0items = nullptr;          // parallel to items: folded c0 source, -1 none (null: no folding)
  int* ownitems = nullptr;         // parallel to items: input ct of the own limbs (null: the item's ct)
  int width = 1;                   // largest group's output count, as a power of two
  std::vector<double> rd, wr;      // host: words per (limb, coefficient) read per digit / written
};
struct KsStage {
  int n_out = 0;
  KipTables batched, single;
  int n_base = 0, n_adds = 0;
  fk::TailItem* tails = nullptr;
  fk::AddTerm* terms = nullptr;
};

// Device tables of a linear-combination stage (classes of outputs with the
// same terms), batched and one output per class.  Classes are ordered by row
// width; a segment is the classes of one width.
struct MacSeg {
  int c0, n, width;
  int ptm;                         // plaintext products: none, one per group, one per (group, output)
  bool diag;                       // every group one term of weight 1 with its own plaintexts
  bool one;                        // every group one weighted term and the class's shared plaintext
  bool fast;                       // every weight code below 2^23 in magnitude
  int chunk;                       // terms per chunk: 8, or 4 for groups of under 6 terms on average
  double words;                    // words per (coefficient, limb) moved by the segment's classes
  double mm;                       // modular products per (coefficient, limb) of the segment's classes
};
struct MacTables {
  int n = 0;                       // classes
  std::vector<MacSeg> seg;
  fk::MacClass* cls = nullptr;
  int* cls_out = nullptr;
  const uint64_t** mask = nullptr;
  int* toff = nullptr;
  int* tin = nullptr;
  d2* ew = nullptr;                // [nl][ews] weight residues
  long long ews = 0;
  double* wc = nullptr;            // [ews] signed codes of the small-code classes
};
struct GmacStage {
  int n_out = 0;
  long long n_terms = 0, n_masked = 0;
  MacTables batched, single;
  // extended basis: limbs Q_l U P (prime indices eprime), A inputs (Q only)
  // weighted by P on the Q limbs and absent on the P limbs
  bool pq = false;
  const unsigned char* eprime = nullptr;
};

struct Plan {
  virtual ~Plan() {
    for (void* p : owned) fb::dev_free(p);
  }
  std::vector<void*> owned;   // device allocations of the plan
  Layout out;
};

struct LevelTabs {
  d2* modup = nullptr;   // [beta][alpha + le*alpha]
  int tstride = 0;
  d2* qlinv = nullptr;   // [level]
  unsigned char* eprime = nullptr;
  std::vector<unsigned char> h_eprime;
  d2* epq = nullptr;     // [le] (q, 1/q) of the prime of extended limb l
  d2* pmod = nullptr;    // [level+1] P mod q_i
  // ModDown by P q_l (level >= 1): per source q_l, p_0 .. p_{K-1}: (D/d_k)^-1 mod d_k,
  // then per limb i < level: (D/d_k) mod q_i; and D^-1 mod q_i
  d2* md_rs = nullptr;
  d2* dinv_rs = nullptr;
  std::vector<uint64_t> h_pmod;
};

}  // namespace fr

struct fenc_ctx {
  fenc_params prm{};
  int logn = 0, N = 0, ns = 0, L = 0, K = 0, alpha = 0, ndig = 0, np = 0;
  double Delta = 1.0;
  std::vector<uint64_t> primes, psi;
  std::vector<int64_t> s;            // secret key coefficients (client role)
  bool has_sk = true;                // false: server context (evaluation keys only)
  int mode = FENC_MODE_BATCHED;
  bool strict = false;
  int64_t pt_budget = 1LL << 30;     // bytes of materialised conv plaintexts (one batch group)
  int64_t own_copy = 1LL << 30;      // extended digits of a stage up to this size get their own limbs copied
  int64_t ws_limit = 32LL << 30;     // workspace per operation; larger batches run in tiles of batch groups
  fenc_counters cnt{};

  // device state (built on first use)
  bool dev = false;
  int device = -1;
  fk::d2 *pq = nullptr, *ninv = nullptr;
  double *tw_fwd = nullptr, *tw_inv = nullptr;
  fk::d2 *md_tab = nullptr, *pinv = nullptr;   // ModDown: hinv[K], hat[L+1][K]; P^-1 mod q_i
  uint64_t* s_ntt = nullptr;                   // [np][N]
  std::map<int, fr::LevelTabs> lvl;
  std::map<uint64_t, uint64_t*> keys;          // Galois element (0: relinearisation) -> key
  std::map<std::string, std::unique_ptr<fr::Plan>> plans;
  std::map<uint64_t, std::vector<int>> maps;
  std::vector<void*> owned;
  fr::Arena arena;
  int64_t dev_bytes = 0;
  std::map<void*, size_t> dev_sizes;          // size of every live allocation made by dalloc
  // NTT pass shapes: [fwd cols, fwd rows, inv rows, inv cols] = {radix bits (3 or 4),
  // log2 of columns (cols pass) or chunks (rows pass) per block}; results do not depend on them
  int ntt_cfg[4][2] = {{3, -1}, {3, -1}, {3, -1}, {3, -1}};
  bool ntt_tuned = false;
  // hoisting schedule of convolutions and S = 1 pooling: 1 = linear
  // combinations of rotated copies in the extended basis with one ModDown per
  // combined ciphertext, 0 = one ModDown per rotated copy
  int hoist = 1;        // hoisting schedule: 0, 1, or 2 (per layer, the smaller modelled traffic)
  int last_hoist = -1;  // schedule of the most recent convolution, pooling or compression
  int baby = 1;         // baby step of convolutions' outer rotations: n >= 1 fixed, 0 chosen per layer
  int last_baby = -1;   // baby step of the most recent convolution
  // single-kernel profiling: events around every launch of `prof_kernel`
  std::string prof_kernel;
  struct ProfRec {
    void *a, *b;
    double bytes;
    double ops;         // algorithmic modular products of the launch(es)
    const char* name;   // kernel name (a string literal)
  };
  std::vector<ProfRec> prof;
  ~fenc_ctx();
};

namespace fr {

typedef fenc_ctx Ctx;

void ensure_device(Ctx& C);
// times the candidate NTT pass shapes on this device and keeps the fastest
void autotune_ntt(Ctx& C);
void* dalloc(Ctx& C, size_t bytes, std::vector<void*>& owner);
// frees every allocation in owner (made by dalloc) and takes it off dev_bytes
void dfree_all(Ctx& C, std::vector<void*>& owner);
template <class T>
T* upload(Ctx& C, const std::vector<T>& v, std::vector<void*>& owner) {
  T* p = (T*)dalloc(C, v.size() * sizeof(T) + 8, owner);
  if (!v.empty()) fb::h2d(p, v.data(), v.size() * sizeof(T));
  return p;
}
const LevelTabs& level_tabs(Ctx& C, int level);
uint64_t galois(const Ctx& C, long long shift);
const uint64_t* get_key(Ctx& C, uint64_t g);
d2 cpair(uint64_t w, uint64_t q);   // (w, w/q)

// NTT of rows: row r reads src + (r/nl)*src_gs + (r%nl)*N, prime pm.p[r % pm.n]
// md or rs (forward only): the row pass ends in that ModDown or rescale tail
// instead of writing dst (md_bytes: the fused row pass's algorithmic bytes);
// lift: the column pass takes its input from that rescale lift instead of src
// (lift_bytes: its algorithmic bytes)
void ntt(Ctx& C, bool inverse, const u64* src, u64* dst, long long src_gs, long long dst_gs, int nrows, int nl,
         const fk::PrimeMap& pm, fb::Stream s, const fk::TailArgs* md = nullptr, double md_bytes = 0,
         const fk::RescaleTailArgs* rs = nullptr, const fk::LiftArgs* lift = nullptr, double lift_bytes = 0);
fk::PrimeMap identity_map(int n);

// key switching pieces
// copy_own: also copy every digit's own limbs into ext (else the KIP reads them from `in`)
void modup(Ctx& C, int level, const u64* in, long long cs, long long ps, int B, u64* ext, fb::Stream s,
           bool copy_own = false);
// Where the key inner product finds the digits' own limbs: with p set, ModUp
// left them out of ext and they are the NTT-form c1 of input ct t at
// p + t * cs, t the item's own input ct (KsItem::own, else the ext ct index);
// with p null they are in ext.
struct ExtOwn {
  const u64* p;
  long long cs;
};


// rs: ModDown by P q_l instead of P, so the outputs (level-1, strides out_cs)
// are (base + KS) / q_l: a relinearisation and its rescale in one conversion
void kip_moddown(Ctx& C, int level, const u64* ext, const ExtOwn& own, const KsStage& st, u64* out, long long out_cs,
                 const u64* base, long long base_cs, const u64* add, long long add_cs, fb::Stream s,
                 bool rs = false);
void rescale(Ctx& C, int level, const u64* in, int B, u64* out, fb::Stream s);
// the rescale with caller-given workspace: last [B][2][N], lift [B][2][level][N]
// (every word is written before it is read)
void rescale_ws(Ctx& C, int level, const u64* in, int B, u64* out, fb::Stream s, u64* last, u64* lift);
size_t rescale_ws_bytes(const Ctx& C, int level, int B);
void run_gmac(Ctx& C, int nl, const GmacStage& g, const u64* in_a, long long a_cs, long long a_ps, int na,
              const u64* in_b, long long b_cs, long long b_ps, u64* out, long long out_cs, long long out_ps,
              fb::Stream s);
// KIP only (no ModDown): acc[o] over Q_l U P in NTT form, with P sigma(c0) folded in
void kip_only(Ctx& C, int level, const u64* ext, const ExtOwn& own, const KsStage& st, u64* acc, const u64* c0, long long c0_cs,
              fb::Stream s);
// ModDown only of n extended-basis ciphertexts acc[o] ([2][le][N], NTT form) into out[o]
void moddown_only(Ctx& C, int level, const u64* acc, const KsStage& md, u64* out, long long out_cs, fb::Stream s);
// out[t] = (P x_t, 0) over Q_l U P for n cts at level (NTT form)
void lift_to_pq(Ctx& C, int level, const u64* in, int n, u64* out, fb::Stream s);
// a ModDown-only stage for n outputs (tails only)
KsStage make_md(Ctx& C, int n, std::vector<void*>& owner);

KsStage make_ks(Ctx& C, const std::vector<std::vector<KsItem>>& items, const std::vector<fk::TailItem>& tails,
                const std::vector<fk::AddTerm>& terms, std::vector<void*>& owner);
struct GmacBuild {
  std::vector<int> goff{0}, toff{0}, tin, tw;
  std::vector<const u64*> mask;
  void add_group(const u64* m) { mask.push_back(m); }
  void add_term(int in, int w) { tin.push_back(in); tw.push_back(w); }
  void end_group() { toff.push_back((int)tin.size()); }
  void end_output() { goff.push_back((int)mask.size()); }
};
GmacStage make_gmac(Ctx& C, const GmacBuild& b, const std::vector<int64_t>& wcodes, int level,
                    std::vector<void*>& owner, bool pq = false, int na = 0);

// plaintexts: encode real slots at `scale`, reduce, NTT on device ([level+1][N])
u64* encode_plaintexts(Ctx& C, const std::vector<std::vector<double>>& slots, double scale, int level,
                       std::vector<void*>& owner, bool ext = false);   // ext: over Q_l U P ([le][N])

int64_t weight_code(double w, double scale);
void split_scale(double T, double& dw, double& dm);

inline long long ct_elems(const Ctx& C, int level) { return 2LL * (level + 1) * C.N; }

// Times the launch(es) issued by `launch` when `name` is the profiled kernel;
// `bytes` is the algorithmic HBM traffic of those launches and `ops` their
// algorithmic modular products (0 where not counted).
// With the profiled name "*" every kernel's launches are timed.
template <class F>
void timed(Ctx& C, const char* name, double bytes, fb::Stream s, F launch, double ops = 0) {
  if (C.prof_kernel.empty() || (C.prof_kernel != "*" && C.prof_kernel != name) || fb::capturing(s)) {
    launch();
    return;
  }
  void* a = fb::event_create();
  void* b = fb::event_create();
  fb::event_record(a, s);
  launch();
  fb::event_record(b, s);
  C.prof.push_back({a, b, bytes, ops, name});
}

}  // namespace fr
