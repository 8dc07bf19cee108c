// Host runtime: device tables, keys, workspace, key-switching pipelines.
//
// Hybrid key switching (the rotation formula of the Background section read
// as Han-Ki hybrid switching with dnum digits):
//   ModUp    iNTT(c1) -> fast base conversion of each digit -> NTT of the new limbs
//   KIP      acc = sum_j sigma_g(ext_j) * key_j        (automorphism fused as a gather)
//   ModDown  iNTT(P limbs) -> base conversion P -> Q -> NTT -> (acc - conv) * P^-1
// Hoisted rotations share one ModUp per input ciphertext; lazy sums share one
// ModDown per output ciphertext.
#include "runtime.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <array>
#include <tuple>
#include <thread>

namespace fr {

using fh::invmod;
using fh::mulmod;

// ---------------------------------------------------------------- arena
Arena::~Arena() {
  for (auto& c : chunks_) fb::dev_free(c.p);
}

void* Arena::get(size_t bytes, fb::Stream s) {
  bytes = (bytes + 255) & ~(size_t)255;
  const bool cap_now = fb::capturing(s);
  if (!chunks_.empty() && off_ + bytes <= chunks_[cur_].cap) {
    void* p = chunks_[cur_].p + off_;
    off_ += bytes;
    chunks_[cur_].pinned = chunks_[cur_].pinned || cap_now;
    return p;
  }
  // the chunks after the current one are free: the first that is large enough
  const size_t from = chunks_.empty() ? 0 : cur_ + 1;
  for (size_t n = from; n < chunks_.size(); n++)
    if (chunks_[n].cap >= bytes) {
      cur_ = n;
      off_ = bytes;
      chunks_[n].pinned = chunks_[n].pinned || cap_now;
      return chunks_[n].p;
    }
  if (cap_now) fail(FENC_ENOMEM, "workspace must grow during stream capture; run the operation once before capturing");
  // return the free chunks that are too small (earlier launches may still use
  // them: wait for the device first), then add one that fits; chunks grow
  // from 64 MiB up to 1 GiB, larger requests get a chunk of their own size
  bool dropped = false;
  for (size_t n = chunks_.size(); n-- > from;)
    if (!chunks_[n].pinned) {
      if (!dropped) fb::device_sync();
      dropped = true;
      fb::dev_free(chunks_[n].p);
      chunks_.erase(chunks_.begin() + n);
    }
  size_t biggest = 0;
  for (auto& c : chunks_) biggest = std::max(biggest, c.cap);
  const size_t grow = chunks_.empty() ? (size_t)64 << 20 : std::min<size_t>(biggest * 2, (size_t)1 << 30);
  const size_t cap = std::max<size_t>(bytes, grow);
  chunks_.push_back({(char*)fb::dev_alloc(cap), cap, false});
  cur_ = chunks_.size() - 1;
  off_ = bytes;
  return chunks_[cur_].p;
}

size_t Arena::bytes() const {
  size_t b = 0;
  for (auto& c : chunks_) b += c.cap;
  return b;
}

// ---------------------------------------------------------------- helpers
d2 cpair(uint64_t w, uint64_t q) { return {(double)w, (double)w / (double)q}; }

void* dalloc(Ctx& C, size_t bytes, std::vector<void*>& owner) {
  void* p = fb::dev_alloc(bytes);
  owner.push_back(p);
  C.dev_bytes += (int64_t)bytes;
  C.dev_sizes[p] = bytes;
  return p;
}

void dfree_all(Ctx& C, std::vector<void*>& owner) {
  for (void* p : owner) {
    auto it = C.dev_sizes.find(p);
    if (it != C.dev_sizes.end()) {
      C.dev_bytes -= (int64_t)it->second;
      C.dev_sizes.erase(it);
    }
    fb::dev_free(p);
  }
  owner.clear();
}

fk::PrimeMap identity_map(int n) {
  fk::PrimeMap pm;
  pm.n = n;
  for (int i = 0; i < n; i++) pm.p[i] = (unsigned char)i;
  return pm;
}

uint64_t galois(const Ctx& C, long long shift) {
  long long r = shift % C.ns;
  if (r < 0) r += C.ns;
  return fh::powmod(5, (uint64_t)r, 2ull * C.N);
}

static unsigned grid_x(const Ctx& C) { return (unsigned)std::max(1, C.N / 256); }
static int block_threads(const Ctx& C) { return std::min(256, C.N); }

// ---------------------------------------------------------------- device set-up
void ensure_device(Ctx& C) {
  if (C.dev) return;
  C.device = fb::device_id();
  const int N = C.N, np = C.np;
  std::vector<d2> pq(np), ni(np);
  std::vector<double> twf((size_t)np * N), twi((size_t)np * N);   // twiddles w (the kernels form w/q)
  for (int p = 0; p < np; p++) {
    const uint64_t q = C.primes[p], psi = C.psi[p], psi_inv = invmod(psi, q);
    pq[p] = {(double)q, 1.0 / (double)q};
    for (int k = 0; k < N; k++) {
      const unsigned e = fh::bitrev((unsigned)k, C.logn);
      twf[(size_t)p * N + k] = (double)fh::powmod(psi, e, q);
      twi[(size_t)p * N + k] = (double)fh::powmod(psi_inv, e, q);
    }
    ni[p] = cpair(invmod((uint64_t)N, q), q);
  }
  C.pq = upload(C, pq, C.owned);
  C.tw_fwd = upload(C, twf, C.owned);
  C.tw_inv = upload(C, twi, C.owned);
  C.ninv = upload(C, ni, C.owned);
  // ModDown tables (level independent): hinv[k] mod p_k, hat[i][k] = (P/p_k) mod q_i, P^-1 mod q_i
  const int K = C.K, L1 = C.L + 1;
  std::vector<d2> md((size_t)K + (size_t)L1 * K), pinv(L1);
  for (int k = 0; k < K; k++) {
    const uint64_t pk = C.primes[L1 + k];
    uint64_t hat = 1;
    for (int k2 = 0; k2 < K; k2++)
      if (k2 != k) hat = mulmod(hat, C.primes[L1 + k2] % pk, pk);
    md[k] = cpair(invmod(hat, pk), pk);
  }
  for (int i = 0; i < L1; i++) {
    const uint64_t qi = C.primes[i];
    uint64_t P = 1;
    for (int k = 0; k < K; k++) {
      uint64_t hat = 1;
      for (int k2 = 0; k2 < K; k2++)
        if (k2 != k) hat = mulmod(hat, C.primes[L1 + k2] % qi, qi);
      md[K + (size_t)i * K + k] = cpair(hat, qi);
      P = mulmod(P, C.primes[L1 + k] % qi, qi);
    }
    pinv[i] = cpair(invmod(P, qi), qi);
  }
  C.md_tab = upload(C, md, C.owned);
  C.pinv = upload(C, pinv, C.owned);
  C.dev = true;
  if (!C.has_sk) {   // a server context: no secret key on the device
    autotune_ntt(C);
    return;
  }
  // secret key in NTT form over every prime
  std::vector<long long> sv(C.s.begin(), C.s.end());
  long long* ds = upload(C, sv, C.owned);
  std::vector<unsigned char> allp(np);
  for (int p = 0; p < np; p++) allp[p] = (unsigned char)p;
  unsigned char* dp = upload(C, allp, C.owned);
  C.s_ntt = (uint64_t*)dalloc(C, (size_t)np * N * 8, C.owned);
  fk::SmallArgs a{ds, C.s_ntt, np, C.logn, dp, C.pq};
  fb::small_to_rns({grid_x(C), (unsigned)np, 1}, block_threads(C), nullptr, a);
  ntt(C, false, C.s_ntt, C.s_ntt, 0, 0, np, np, identity_map(np), nullptr);
  fb::sync(nullptr);
  autotune_ntt(C);
}

const LevelTabs& level_tabs(Ctx& C, int level) {
  auto it = C.lvl.find(level);
  if (it != C.lvl.end()) return it->second;
  LevelTabs T;
  const int nl = level + 1, le = nl + C.K, alpha = C.alpha, beta = (nl + alpha - 1) / alpha;
  T.h_eprime.resize(le);
  for (int l = 0; l < le; l++) T.h_eprime[l] = (unsigned char)(l < nl ? l : C.L + 1 + (l - nl));
  T.eprime = upload(C, T.h_eprime, C.owned);
  std::vector<d2> epq(le);
  for (int l = 0; l < le; l++) {
    const uint64_t q = C.primes[T.h_eprime[l]];
    epq[l] = {(double)q, 1.0 / (double)q};
  }
  T.epq = upload(C, epq, C.owned);
  T.tstride = alpha + le * alpha;
  std::vector<d2> tab((size_t)beta * T.tstride, d2{0, 0});
  for (int j = 0; j < beta; j++) {
    const int lo = j * alpha, hi = std::min(lo + alpha, nl);
    d2* t = &tab[(size_t)j * T.tstride];
    for (int i = lo; i < hi; i++) {
      const uint64_t qi = C.primes[i];
      uint64_t hat = 1;
      for (int i2 = lo; i2 < hi; i2++)
        if (i2 != i) hat = mulmod(hat, C.primes[i2] % qi, qi);
      t[i - lo] = cpair(invmod(hat, qi), qi);
    }
    for (int l = 0; l < le; l++) {
      if (l >= lo && l < hi) continue;
      const uint64_t qt = C.primes[T.h_eprime[l]];
      for (int i = lo; i < hi; i++) {
        uint64_t hat = 1;
        for (int i2 = lo; i2 < hi; i2++)
          if (i2 != i) hat = mulmod(hat, C.primes[i2] % qt, qt);
        t[alpha + (size_t)l * alpha + (i - lo)] = cpair(hat, qt);
      }
    }
  }
  T.modup = upload(C, tab, C.owned);
  std::vector<d2> ql(std::max(1, level));
  for (int i = 0; i < level; i++) ql[i] = cpair(invmod(C.primes[level] % C.primes[i], C.primes[i]), C.primes[i]);
  T.qlinv = upload(C, ql, C.owned);
  std::vector<d2> pm(nl);
  T.h_pmod.resize(nl);
  for (int i = 0; i < nl; i++) {
    uint64_t P = 1;
    for (int k = 0; k < C.K; k++) P = mulmod(P, C.primes[C.L + 1 + k] % C.primes[i], C.primes[i]);
    T.h_pmod[i] = P;
    pm[i] = cpair(P, C.primes[i]);
  }
  T.pmod = upload(C, pm, C.owned);
  if (level >= 1) {   // ModDown by D = P q_l: sources q_l, p_0 .. p_{K-1}
    const int K1 = C.K + 1;
    std::vector<uint64_t> dp(K1);
    dp[0] = C.primes[level];
    for (int k = 0; k < C.K; k++) dp[k + 1] = C.primes[C.L + 1 + k];
    std::vector<d2> rs((size_t)K1 + (size_t)level * K1), dinv(level);
    for (int k = 0; k < K1; k++) {
      uint64_t hat = 1;
      for (int k2 = 0; k2 < K1; k2++)
        if (k2 != k) hat = mulmod(hat, dp[k2] % dp[k], dp[k]);
      rs[k] = cpair(invmod(hat, dp[k]), dp[k]);
    }
    for (int i = 0; i < level; i++) {
      const uint64_t qi = C.primes[i];
      uint64_t D = 1;
      for (int k = 0; k < K1; k++) {
        uint64_t hat = 1;
        for (int k2 = 0; k2 < K1; k2++)
          if (k2 != k) hat = mulmod(hat, dp[k2] % qi, qi);
        rs[K1 + (size_t)i * K1 + k] = cpair(hat, qi);
        D = mulmod(D, dp[k] % qi, qi);
      }
      dinv[i] = cpair(invmod(D, qi), qi);
    }
    T.md_rs = upload(C, rs, C.owned);
    T.dinv_rs = upload(C, dinv, C.owned);
  }
  return C.lvl[level] = T;
}

// ---------------------------------------------------------------- NTT
void ntt(Ctx& C, bool inverse, const u64* src, u64* dst, long long src_gs, long long dst_gs, int nrows, int nl,
         const fk::PrimeMap& pm, fb::Stream s, const fk::TailArgs* md, double md_bytes,
         const fk::RescaleTailArgs* rs, const fk::LiftArgs* lift, double lift_bytes) {
  if (nrows <= 0) return;
  fk::NttArgs a;
  a.src = src;
  a.dst = dst;
  a.src_gs = src_gs;
  a.dst_gs = dst_gs;
  a.nrows = nrows;
  a.nl = nl;
  a.pm = pm;
  a.tw = inverse ? C.tw_inv : C.tw_fwd;
  a.pq = C.pq;
  a.ninv = C.ninv;
  a.logn = C.logn;
  a.n2 = (C.logn + 1) / 2;
  a.n1 = C.logn - a.n2;
  // pass shape: radix bits and tile (defaults: radix 8, 16 columns / ~2048 elements per block)
  auto shape = [&](int k, int P, int other, int def) {
    const int rb = C.ntt_cfg[k][0];
    const int t = C.ntt_cfg[k][1] >= 0 ? std::min(C.ntt_cfg[k][1], other) : def;
    const int nr = (P + rb - 1) / rb, kmax = P / nr + (P % nr ? 1 : 0);   // size of the first (largest) round
    const int T = (int)std::min<long long>(256, std::max<long long>(64, 1LL << std::max(0, P + t - kmax)));
    return std::array<int, 3>{rb, t, T};
  };
  const auto fc = shape(inverse ? 3 : 0, a.n1, a.n2, std::min(4, a.n2));
  const auto fr = shape(inverse ? 2 : 1, a.n2, a.n1, std::min(std::max(0, 11 - a.n2), a.n1));
  a.lcols = fc[1];
  a.lcpb = fr[1];
  const unsigned colblocks = 1u << (a.n2 - a.lcols), rowblocks = 1u << (a.n1 - a.lcpb);
  // LDS: the tile (column pass: then its 2^n1 twiddles)
  const size_t lds_c = ((size_t)8 << (a.n1 + a.lcols)) + ((size_t)8 << a.n1);
  const size_t lds_r = (size_t)8 << (a.n2 + a.lcpb);
  int active = 0;
  for (int r = 0; r < std::min(nrows, pm.n); r++) active += (pm.p[r] != fk::kSkip);
  active = (int)((long long)active * nrows / std::max(1, std::min(nrows, pm.n)));
  const double pass_bytes = 16.0 * active * C.N;   // read + write of every active row
  // modular products: one per butterfly (N/2 per stage and row); the inverse
  // column pass also scales by 1/N, the ModDown and rescale tails multiply
  // every output word by P^-1 or q_l^-1
  const double ops_c = 0.5 * active * C.N * a.n1, ops_r = 0.5 * active * C.N * a.n2;
  const fb::Grid gc{colblocks, (unsigned)nrows, 1}, gr{rowblocks, (unsigned)nrows, 1};
  if (!inverse) {
    if (lift) {   // the column pass starts from the rescale lift
      const fk::NttLiftArgs m{a, *lift};
      timed(C, "ntt_fwd_cols_lift", lift_bytes, s, [&] {
        if (fc[0] == 4) fb::ntt_fwd_cols16_lift(gc, fc[2], lds_c, s, m);
        else fb::ntt_fwd_cols_lift(gc, fc[2], lds_c, s, m);
      }, ops_c);
    } else {
      timed(C, "ntt_fwd_cols", pass_bytes, s, [&] {
        if (fc[0] == 4) fb::ntt_fwd_cols16(gc, fc[2], lds_c, s, a);
        else fb::ntt_fwd_cols(gc, fc[2], lds_c, s, a);
      }, ops_c);
    }
    a.src = dst;
    a.src_gs = dst_gs;
    if (md) {   // the row pass ends in the ModDown tail
      const fk::NttMdArgs m{a, *md};
      timed(C, "ntt_fwd_rows_md", md_bytes, s, [&] {
        if (fr[0] == 4) fb::ntt_fwd_rows16_md(gr, fr[2], lds_r, s, m);
        else fb::ntt_fwd_rows_md(gr, fr[2], lds_r, s, m);
      }, ops_r + (double)active * C.N);
    } else if (rs) {   // the row pass ends in the rescale tail
      const fk::NttRsArgs m{a, *rs};
      timed(C, "ntt_fwd_rows_rs", md_bytes, s, [&] {
        if (fr[0] == 4) fb::ntt_fwd_rows16_rs(gr, fr[2], lds_r, s, m);
        else fb::ntt_fwd_rows_rs(gr, fr[2], lds_r, s, m);
      }, ops_r + (double)active * C.N);
    } else {
      timed(C, "ntt_fwd_rows", pass_bytes, s, [&] {
        if (fr[0] == 4) fb::ntt_fwd_rows16(gr, fr[2], lds_r, s, a);
        else fb::ntt_fwd_rows(gr, fr[2], lds_r, s, a);
      }, ops_r);
    }
    C.cnt.ntt_limbs += active;
  } else {
    timed(C, "ntt_inv_rows", pass_bytes, s, [&] {
      if (fr[0] == 4) fb::ntt_inv_rows16(gr, fr[2], lds_r, s, a);
      else fb::ntt_inv_rows(gr, fr[2], lds_r, s, a);
    }, ops_r);
    a.src = dst;
    a.src_gs = dst_gs;
    timed(C, "ntt_inv_cols", pass_bytes, s, [&] {
      if (fc[0] == 4) fb::ntt_inv_cols16(gc, fc[2], lds_c, s, a);
      else fb::ntt_inv_cols(gc, fc[2], lds_c, s, a);
    }, ops_c + (double)active * C.N);
    C.cnt.intt_limbs += active;
  }
  C.cnt.launches += 2;
}

// ---------------------------------------------------------------- NTT autotuning
// Every candidate pass shape computes the same residues; only speed differs.
// Each pass is timed on a batch of rows with HIP events and the fastest shape
// is kept.  Skipped on the CPU emulator and while a stream is being captured.
void autotune_ntt(Ctx& C) {
  if (C.ntt_tuned) return;
  C.ntt_tuned = true;
  if (std::string(fb::backend_name()) != "hip-gfx950" || C.logn < 10 || fb::capturing(nullptr)) return;
  const int rows = std::max(8, std::min(256, (int)((64LL << 20) / ((long long)C.N * 8))));
  std::vector<void*> tmp;
  u64* buf = (u64*)dalloc(C, (size_t)rows * C.N * 8, tmp);
  std::vector<u64> zero((size_t)C.N, 0);
  for (int r = 0; r < rows; r++) fb::h2d(buf + (size_t)r * C.N, zero.data(), (size_t)C.N * 8);
  fk::PrimeMap pm;
  pm.n = std::min(C.np, fk::kMaxMap);
  for (int i = 0; i < pm.n; i++) pm.p[i] = (unsigned char)i;
  const int n2 = (C.logn + 1) / 2, n1 = C.logn - n2;
  void* e0 = fb::event_create();
  void* e1 = fb::event_create();
  auto time_dir = [&](bool inverse) {
    float best = 0;
    fb::sync(nullptr);
    for (int rep = 0; rep < 4; rep++) {
      fb::event_record(e0, nullptr);
      ntt(C, inverse, buf, buf, (long long)pm.n * C.N, (long long)pm.n * C.N, rows, pm.n, pm, nullptr);
      fb::event_record(e1, nullptr);
      const float ms = fb::event_elapsed_ms(e0, e1);
      if (rep > 0 && (best == 0 || ms < best)) best = ms;
    }
    return best;
  };
  // tune one pass at a time, the other pass at its current shape
  for (int k = 0; k < 4; k++) {
    const bool inverse = k >= 2, cols = (k == 0 || k == 3);
    const int P = cols ? n1 : n2, other = cols ? n2 : n1;
    int best_rb = C.ntt_cfg[k][0], best_t = C.ntt_cfg[k][1];
    float best = time_dir(inverse);
    for (int rb = 3; rb <= 4; rb++)
      for (int t = 0; t <= std::min(other, 5); t++) {
        if ((8LL << (P + t)) > (64 << 10)) continue;   // LDS tile (without twiddles) at most 64 KiB
        if ((1LL << (P + t)) < 512) continue;         // at least 512 elements per block
        C.ntt_cfg[k][0] = rb;
        C.ntt_cfg[k][1] = t;
        const float ms = time_dir(inverse);
        if (ms < best) {
          best = ms;
          best_rb = rb;
          best_t = t;
        }
      }
    C.ntt_cfg[k][0] = best_rb;
    C.ntt_cfg[k][1] = best_t;
  }
  fb::sync(nullptr);
  fb::event_destroy(e0);
  fb::event_destroy(e1);
  dfree_all(C, tmp);
}

// ---------------------------------------------------------------- keys
const uint64_t* get_key(Ctx& C, uint64_t g) {
  auto it = C.keys.find(g);
  if (it != C.keys.end()) return it->second;
  if (C.strict) fail(FENC_ENOKEY, "missing switching key for Galois element " + std::to_string(g));
  if (!C.has_sk)
    fail(FENC_ENOKEY, "server context holds no secret key: import the switching key for Galois element " +
                          std::to_string(g));
  ensure_device(C);
  const int N = C.N, np = C.np, nd = C.ndig, L1 = C.L + 1;
  const uint64_t seed = C.prm.seed;
  // host sampling of the uniform a_j and the errors e_j
  std::vector<uint64_t> a((size_t)nd * np * N);
  std::vector<long long> e((size_t)nd * N);
  const int nthr = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  for (int w = 0; w < nthr; w++)
    th.emplace_back([&, w] {
      for (int r = w; r < nd * np; r += nthr) {
        const int j = r / np, p = r % np;
        const uint64_t q = C.primes[p], tg = fh::tag::key_a(g, j, p);
        uint64_t* dst = &a[(size_t)r * N];
        for (int i = 0; i < N; i++) dst[i] = fh::draw_uniform(seed, tg, i, q);
      }
      for (int j = w; j < nd; j += nthr)
        for (int i = 0; i < N; i++) e[(size_t)j * N + i] = fh::draw_gauss(seed, fh::tag::key_e(g, j), i);
    });
  for (auto& t : th) t.join();
  std::vector<void*> tmp;
  uint64_t* da = upload(C, a, tmp);
  long long* de = upload(C, e, tmp);
  std::vector<unsigned char> allp(np);
  for (int p = 0; p < np; p++) allp[p] = (unsigned char)p;
  unsigned char* dp = upload(C, allp, tmp);
  uint64_t* dE = (uint64_t*)dalloc(C, (size_t)nd * np * N * 8, tmp);
  uint64_t* dS = (uint64_t*)dalloc(C, (size_t)np * N * 8, tmp);
  ntt(C, false, da, da, (long long)np * N, (long long)np * N, nd * np, np, identity_map(np), nullptr);
  fk::SmallArgs sa{de, dE, np, C.logn, dp, C.pq};
  fb::small_to_rns({grid_x(C), (unsigned)(nd * np), 1}, block_threads(C), nullptr, sa);
  ntt(C, false, dE, dE, (long long)np * N, (long long)np * N, nd * np, np, identity_map(np), nullptr);
  fk::PermArgs pa{C.s_ntt, dS, (unsigned)g, C.logn, dp, C.pq};   // g == 0: s^2, else sigma_g(s)
  fb::perm_rows({grid_x(C), (unsigned)np, 1}, block_threads(C), nullptr, pa);
  std::vector<d2> gad((size_t)nd * np, d2{0, 0});
  for (int j = 0; j < nd; j++)
    for (int p = j * C.alpha; p < std::min((j + 1) * C.alpha, L1); p++) {
      uint64_t P = 1;
      for (int k = 0; k < C.K; k++) P = mulmod(P, C.primes[L1 + k] % C.primes[p], C.primes[p]);
      gad[(size_t)j * np + p] = cpair(P, C.primes[p]);
    }
  d2* dg = upload(C, gad, tmp);
  uint64_t* key = (uint64_t*)dalloc(C, (size_t)nd * 2 * np * N * 8, C.owned);
  fk::KeyArgs ka{da, dE, C.s_ntt, dS, key, dg, np, C.logn, C.pq};
  fb::key_combine({grid_x(C), (unsigned)(nd * np), 1}, block_threads(C), nullptr, ka);
  fb::sync(nullptr);
  dfree_all(C, tmp);
  C.keys[g] = key;
  return key;
}

// ---------------------------------------------------------------- key switching
void modup(Ctx& C, int level, const u64* in, long long cs, long long ps, int B, u64* ext, fb::Stream s,
           bool copy_own) {
  if (B <= 0) return;
  const LevelTabs& T = level_tabs(C, level);
  const int nl = level + 1, le = nl + C.K, beta = (nl + C.alpha - 1) / C.alpha, N = C.N;
  if (beta * le > fk::kMaxMap) fail(FENC_EUNSUPPORTED, "too many extended limbs");
  Scope sc(C.arena);
  u64* coef = (u64*)C.arena.get((size_t)B * nl * N * 8, s);
  fk::PrimeMap pmd;
  pmd.n = beta * le;
  for (int j = 0; j < beta; j++)
    for (int l = 0; l < le; l++) {
      const bool own = l >= j * C.alpha && l < std::min((j + 1) * C.alpha, nl);
      pmd.p[j * le + l] = own ? fk::kSkip : T.h_eprime[l];
    }
  fk::ModUpArgs a;
  a.coef = coef;
  a.coef_cs = (long long)nl * N;
  a.ntt = copy_own ? in + ps : nullptr;
  a.ntt_cs = cs;
  a.ext = ext;
  a.beta = beta;
  a.alpha = C.alpha;
  a.nl = nl;
  a.le = le;
  a.logn = C.logn;
  a.epq = T.epq;
  a.tab = T.modup;
  a.tstride = T.tstride;
  const bool per_op = C.mode == FENC_MODE_PER_OP;
  for (int b0 = 0; b0 < B; b0 += per_op ? 1 : B) {
    const int nb = per_op ? 1 : B;
    ntt(C, true, in + ps + b0 * cs, coef + (long long)b0 * nl * N, cs, (long long)nl * N, nb * nl, nl,
        identity_map(nl), s);
    a.b0 = b0;
    double mb = 0, mo = 0;
    for (int j = 0; j < beta; j++) {
      const int aj = std::min((j + 1) * C.alpha, nl) - j * C.alpha;
      mb += (copy_own ? 2.0 * aj + le : (double)le) * N * 8.0;   // the digit's limbs read (and copied), the rest written
      mo += (double)aj * (1 + (le - aj)) * N;   // y_i, then one product per (source, target) limb
    }
    timed(C, "modup_fbc", mb * nb, s,
          [&] { fb::modup_fbc({(unsigned)(N / block_threads(C)), (unsigned)(nb * beta), 1}, block_threads(C), s, a); },
          mo * nb);
    ntt(C, false, ext + (long long)b0 * beta * le * N, ext + (long long)b0 * beta * le * N, (long long)le * N,
        (long long)le * N, nb * beta * le, le, pmd, s);
    C.cnt.launches += 1;
    C.cnt.modup += nb;
  }
}

// ModDown of outputs o0 .. o0+no-1 of acc ([n][2][le][N], NTT form; its P
// limbs are transformed in place), then the tail into out
// rs: ModDown by P q_l (sources q_l and the special primes, outputs the
// level-1 limbs); the q_l limb of acc first takes P base (rs_prep)
static void moddown_part(Ctx& C, int level, u64* acc, u64* conv, const KsStage& st, int o0, int no, u64* out,
                         long long out_cs, const u64* base, long long base_cs, const u64* add, long long add_cs,
                         fb::Stream s, bool rs = false) {
  const LevelTabs& T = level_tabs(C, level);
  const int nl = level + 1, le = nl + C.K, N = C.N;
  const int nk = rs ? C.K + 1 : C.K, no_l = rs ? nl - 1 : nl;   // converted limbs, output limbs
  if (rs && (level < 1 || !base)) fail(FENC_EINVAL, "ModDown by P q_l needs a level and a base");
  fk::PrimeMap pmP;
  pmP.n = le;
  for (int l = 0; l < le; l++) pmP.p[l] = l < no_l ? fk::kSkip : T.h_eprime[l];
  u64* acc0 = acc + (long long)o0 * 2 * le * N;
  if (rs) {
    const fk::RsPrepArgs r{acc, base, base_cs, (long long)nl * N, st.tails, o0, nl, le, C.logn,
                           cpair(T.h_pmod[nl - 1], C.primes[nl - 1]),
                           d2{(double)C.primes[nl - 1], 1.0 / (double)C.primes[nl - 1]}};
    timed(C, "rs_prep", 3.0 * 2 * no * N * 8, s, [&] {
      fb::rs_prep({(unsigned)(N / block_threads(C)), (unsigned)(2 * no), 1}, block_threads(C), s, r);
    }, 2.0 * no * N);
  }
  ntt(C, true, acc0, acc0, (long long)le * N, (long long)le * N, no * 2 * le, le, pmP, s);
  fk::ModDownArgs m{acc, conv, o0, no_l, le, nk, C.logn, T.epq, rs ? T.md_rs : C.md_tab};
  timed(C, "moddown_fbc", 2.0 * no * (nk + no_l) * N * 8, s, [&] {
    fb::moddown_fbc({(unsigned)(N / block_threads(C)), (unsigned)(2 * no), 1}, block_threads(C), s, m);
  }, 2.0 * no * nk * (1.0 + no_l) * N);
  u64* conv0 = conv + (long long)o0 * 2 * no_l * N;
  fk::TailArgs t;
  t.acc = acc;
  t.conv = conv;
  t.items = st.tails;
  t.terms = st.terms;
  t.o0 = o0;
  t.nl = no_l;
  t.le = le;
  t.logn = C.logn;
  t.out = out;
  t.out_cs = out_cs;
  t.out_ps = (long long)no_l * N;
  t.base = base;
  t.base_cs = base_cs;
  t.base_ps = (long long)nl * N;
  t.add = add;
  t.add_cs = add_cs;
  t.pinv = rs ? T.dinv_rs : C.pinv;
  t.pq = C.pq;
  t.bscale = rs ? T.qlinv : nullptr;   // (P base_i) / (P q_l) = base_i q_l^-1
  // NTT of the converted values; its row pass applies the tail: reads the
  // converted words and acc, writes the output (plus base and added words)
  const double frac = (double)no / st.n_out;
  const double tb = (6.0 * no + 2.0 * st.n_base * frac + st.n_adds * frac) * no_l * N * 8;
  ntt(C, false, conv0, conv0, (long long)no_l * N, (long long)no_l * N, no * 2 * no_l, no_l, identity_map(no_l), s,
      &t, tb);
  C.cnt.launches += 1;
  C.cnt.moddown += no;
  if (rs) C.cnt.rescale += no;
}

static void kip_launch(Ctx& C, int level, const u64* ext, const ExtOwn& own, const KsStage& st, int it, u64* acc,
                       const u64* c0, long long c0_cs, fb::Stream s) {
  const LevelTabs& T = level_tabs(C, level);
  const int nl = level + 1, le = nl + C.K, beta = (nl + C.alpha - 1) / C.alpha, N = C.N;
  const bool per_op = C.mode == FENC_MODE_PER_OP;
  const KipTables& KT = per_op ? st.single : st.batched;
  const int g0 = per_op ? it : 0, ng = per_op ? 1 : KT.n;
  fk::KipArgs k{ext, acc, KT.groups, KT.keys, KT.items, g0, beta, le, C.logn, C.np, T.eprime, C.pq,
                nullptr, nullptr, 0, nullptr, nl, per_op ? 1 : KT.width, own.p, own.cs, KT.ownitems, C.alpha};
  if (c0 && KT.c0items) {
    k.c0ct = KT.c0items;
    k.c0 = c0;
    k.c0_cs = c0_cs;
    k.pmod = T.pmod;
  }
  double kb = 0, ko = 0;
  for (int g = g0; g < g0 + ng; g++) {
    kb += KT.rd[g] * beta + KT.wr[g];
    ko += KT.wr[g] * beta;   // each output word: one product per digit
  }
  kb *= (double)le * N * 8;
  timed(C, "kip", kb, s,
        [&] {   // a thread per coefficient pair
          const int kt = std::min(256, N / 2);
          if (own.p) fb::kip_own({(unsigned)(N / 2 / kt), (unsigned)le, (unsigned)ng}, kt, s, k);
          else fb::kip({(unsigned)(N / 2 / kt), (unsigned)le, (unsigned)ng}, kt, s, k);
        }, ko * le * N);
  C.cnt.launches += 1;
}

void kip_moddown(Ctx& C, int level, const u64* ext, const ExtOwn& own, const KsStage& st, u64* out, long long out_cs,
                 const u64* base, long long base_cs, const u64* add, long long add_cs, fb::Stream s, bool rs) {
  if (st.n_out <= 0) return;
  const int nl = level + 1, le = nl + C.K, N = C.N;
  Scope sc(C.arena);
  const bool per_op = C.mode == FENC_MODE_PER_OP;
  u64* acc = (u64*)C.arena.get((size_t)st.n_out * 2 * le * N * 8, s);
  u64* conv = (u64*)C.arena.get((size_t)st.n_out * 2 * nl * N * 8, s);
  // per-op: one launch sequence per output; batched: every output at once
  const int steps = per_op ? st.n_out : 1;
  for (int it = 0; it < steps; it++) {
    kip_launch(C, level, ext, own, st, it, acc, nullptr, 0, s);
    moddown_part(C, level, acc, conv, st, per_op ? it : 0, per_op ? 1 : st.n_out, out, out_cs, base, base_cs, add,
                 add_cs, s, rs);
  }
}

void kip_only(Ctx& C, int level, const u64* ext, const ExtOwn& own, const KsStage& st, u64* acc, const u64* c0,
              long long c0_cs,
              fb::Stream s) {
  if (st.n_out <= 0) return;
  const int steps = C.mode == FENC_MODE_PER_OP ? st.n_out : 1;
  for (int it = 0; it < steps; it++) kip_launch(C, level, ext, own, st, it, acc, c0, c0_cs, s);
}

void moddown_only(Ctx& C, int level, const u64* acc, const KsStage& md, u64* out, long long out_cs, fb::Stream s) {
  if (md.n_out <= 0) return;
  const int nl = level + 1;
  Scope sc(C.arena);
  u64* conv = (u64*)C.arena.get((size_t)md.n_out * 2 * nl * C.N * 8, s);
  const bool per_op = C.mode == FENC_MODE_PER_OP;
  const int steps = per_op ? md.n_out : 1;
  for (int it = 0; it < steps; it++)
    moddown_part(C, level, (u64*)acc, conv, md, per_op ? it : 0, per_op ? 1 : md.n_out, out, out_cs, nullptr, 0,
                 nullptr, 0, s);
}

void lift_to_pq(Ctx& C, int level, const u64* in, int n, u64* out, fb::Stream s) {
  if (n <= 0) return;
  const LevelTabs& T = level_tabs(C, level);
  const int nl = level + 1, le = nl + C.K;
  const bool per_op = C.mode == FENC_MODE_PER_OP;
  for (int b0 = 0; b0 < n; b0 += per_op ? 1 : n) {
    const int nb = per_op ? 1 : n;
    fk::LiftPqArgs a{in + (long long)b0 * 2 * nl * C.N, 2LL * nl * C.N, out + (long long)b0 * 2 * le * C.N,
                     2LL * le * C.N, nl, le, C.logn, T.pmod, C.pq};
    timed(C, "lift_pq", 2.0 * nb * (nl + le) * C.N * 8, s, [&] {
      fb::lift_pq({(unsigned)(C.N / block_threads(C)), (unsigned)(2 * le), (unsigned)nb}, block_threads(C), s, a);
    });
    C.cnt.launches++;
  }
}

KsStage make_md(Ctx& C, int n, std::vector<void*>& owner) {
  std::vector<fk::TailItem> tails;
  for (int o = 0; o < n; o++) tails.push_back(fk::TailItem{o, -1, 0, 0});
  KsStage st;
  st.n_out = n;
  st.tails = upload(C, tails, owner);
  st.terms = nullptr;
  return st;
}

void rescale(Ctx& C, int level, const u64* in, int B, u64* out, fb::Stream s) {
  if (B <= 0) return;
  if (level < 1) fail(FENC_ELEVEL, "no level left to rescale");
  Scope sc(C.arena);
  u64* last = (u64*)C.arena.get((size_t)B * 2 * C.N * 8, s);
  u64* lift = (u64*)C.arena.get((size_t)B * 2 * level * C.N * 8, s);
  rescale_ws(C, level, in, B, out, s, last, lift);
}

size_t rescale_ws_bytes(const Ctx& C, int level, int B) { return (size_t)B * 2 * (1 + level) * C.N * 8; }

void rescale_ws(Ctx& C, int level, const u64* in, int B, u64* out, fb::Stream s, u64* last, u64* lift) {
  const LevelTabs& T = level_tabs(C, level);
  const int nl = level, N = C.N;   // output limbs
  fk::PrimeMap pl;
  pl.n = 1;
  pl.p[0] = (unsigned char)level;
  const bool per_op = C.mode == FENC_MODE_PER_OP;
  for (int b0 = 0; b0 < B; b0 += per_op ? 1 : B) {
    const int nb = per_op ? 1 : B;
    const long long in_cs = 2LL * (level + 1) * N, out_cs = 2LL * nl * N;
    ntt(C, true, in + b0 * in_cs + (long long)level * N, last + (long long)b0 * 2 * N, (long long)(level + 1) * N,
        N, nb * 2, 1, pl, s);
    // NTT of the last limb lifted to every other limb: the column pass lifts
    // as it loads (reads the last limb, writes the lifted rows' first pass),
    // the row pass applies the tail (reads them and the input, writes the output)
    u64* l0 = lift + (long long)b0 * 2 * nl * N;
    fk::LiftArgs la{last + (long long)b0 * 2 * N, nl, C.logn, (double)C.primes[level], C.pq};
    fk::RescaleTailArgs ra{in + b0 * in_cs, l0, out + b0 * out_cs, nl, C.logn, T.qlinv, C.pq};
    ntt(C, false, l0, l0, (long long)nl * N, (long long)nl * N, nb * 2 * nl, nl, identity_map(nl), s, nullptr,
        6.0 * nb * nl * N * 8, &ra, &la, (2.0 * nb + 2.0 * nb * nl) * N * 8);
    C.cnt.rescale += nb;
  }
}

void run_gmac(Ctx& C, int nl, const GmacStage& g, const u64* in_a, long long a_cs, long long a_ps, int na,
              const u64* in_b, long long b_cs, long long b_ps, u64* out, long long out_cs, long long out_ps,
              fb::Stream s) {
  if (g.n_out <= 0) return;
  const bool per_op = C.mode == FENC_MODE_PER_OP;
  const MacTables& M = per_op ? g.single : g.batched;
  // extended basis: nl Q limbs of the A inputs, nl + K limbs processed
  const int nlimbs = g.pq ? nl + C.K : nl;
  fk::GmacArgs a;
  a.in_a = in_a;
  a.a_cs = a_cs;
  a.a_ps = a_ps;
  a.na = na;
  a.in_b = in_b;
  a.b_cs = b_cs;
  a.b_ps = b_ps;
  a.nl_a = nl;
  a.out = out;
  a.out_cs = out_cs;
  a.out_ps = out_ps;
  a.cls = M.cls;
  a.cls_out = M.cls_out;
  a.mask = M.mask;
  a.toff = M.toff;
  a.tin = M.tin;
  a.ew = M.ew;
  a.ews = M.ews;
  a.wc = M.wc;
  a.nl = nlimbs;
  a.logn = C.logn;
  a.eprime = g.pq ? g.eprime : nullptr;
  a.pq = C.pq;
  nl = nlimbs;
  // batched: one launch per class width; per-op: one launch per class (width 1)
  for (const MacSeg& sg : M.seg) {
    const int steps = per_op ? sg.n : 1;
    for (int it = 0; it < steps; it++) {
      a.c0 = sg.c0 + (per_op ? it : 0);
      a.width = sg.width;
      a.chunk = sg.chunk;
      const int nc = per_op ? 1 : sg.n;
      const double gb = sg.words / sg.n * nc * nl * C.N * 8, go = sg.mm / sg.n * nc * nl * C.N;
      const fb::Grid grid{(unsigned)(C.N / block_threads(C)), (unsigned)nl, (unsigned)(2 * nc)};
      static const char* const names[2][3] = {{"gmac", "gmac_pt", "gmac_ptv"},
                                                {"gmac_fast", "gmac_pt_fast", "gmac_ptv_fast"}};
      typedef void (*Launch)(fb::Grid, int, fb::Stream, const fk::GmacArgs&);
      static const Launch launch[2][3] = {{fb::gmac, fb::gmac_pt, fb::gmac_ptv},
                                          {fb::gmac_fast, fb::gmac_pt_fast, fb::gmac_ptv_fast}};
      const char* name = sg.diag ? "gmac_diag" : sg.one ? "gmac_one" : names[sg.fast][sg.ptm];
      const Launch fn = sg.diag ? fb::gmac_diag : sg.one ? fb::gmac_one : launch[sg.fast][sg.ptm];
      timed(C, name, gb, s, [&] { fn(grid, block_threads(C), s, a); }, go);
      C.cnt.launches += 1;
    }
  }
}

static KipTables make_kip_tables(Ctx& C, const std::vector<std::vector<KsItem>>& items, bool single,
                                 std::vector<void*>& owner) {
  // batched: consecutive outputs with the same ordered key list share a group
  std::vector<fk::KipGroup> groups;
  std::vector<fk::KipKey> keys;
  std::vector<int> it, c0it, ownit;
  bool any_c0 = false, any_own = false;
  std::vector<double> bytes, wbytes;
  const int n = (int)items.size();
  int o = 0;
  while (o < n) {
    int e = o + 1;
    if (!single)
      while (e < n && e - o < fk::kKipOut && items[e].size() == items[o].size()) {
        bool same = true;
        for (size_t k = 0; k < items[o].size(); k++) same = same && items[e][k].g == items[o][k].g;
        if (!same) break;
        e++;
      }
    fk::KipGroup G{o, e - o, (int)keys.size(), (int)items[o].size()};
    for (size_t k = 0; k < items[o].size(); k++) {
      keys.push_back(fk::KipKey{items[o][k].g, items[o][k].key, (int)it.size()});
      for (int oo = o; oo < o + fk::kKipOut; oo++) {
        it.push_back(oo < e ? items[oo][k].ct : -1);
        c0it.push_back(oo < e ? items[oo][k].c0ct : -1);
        any_c0 = any_c0 || (oo < e && items[oo][k].c0ct >= 0);
        // padded slots: input ct 0, which exists
        ownit.push_back(oo < e ? (items[oo][k].own >= 0 ? items[oo][k].own : items[oo][k].ct) : 0);
        any_own = any_own || (oo < e && items[oo][k].own >= 0);
      }
    }
    // words per (limb, coefficient): per digit, nkey keys (2 words) and one ext word per item
    bytes.push_back((double)items[o].size() * ((e - o) + 2));
    wbytes.push_back(2.0 * (e - o));
    groups.push_back(G);
    o = e;
  }
  KipTables T;
  T.n = (int)groups.size();
  for (auto& g : groups)
    while (T.width < g.nout) T.width *= 2;
  T.groups = upload(C, groups, owner);
  T.keys = upload(C, keys, owner);
  T.items = upload(C, it, owner);
  if (any_c0) T.c0items = upload(C, c0it, owner);
  if (any_own) T.ownitems = upload(C, ownit, owner);
  T.rd = bytes;
  T.wr = wbytes;
  return T;
}

KsStage make_ks(Ctx& C, const std::vector<std::vector<KsItem>>& items, const std::vector<fk::TailItem>& tails,
                const std::vector<fk::AddTerm>& terms, std::vector<void*>& owner) {
  KsStage st;
  st.n_out = (int)items.size();
  st.batched = make_kip_tables(C, items, false, owner);
  st.single = make_kip_tables(C, items, true, owner);
  for (auto& t : tails) {
    st.n_base += t.base >= 0;
    st.n_adds += t.add_n;
  }
  st.tails = upload(C, tails, owner);
  st.terms = upload(C, terms, owner);
  return st;
}

static MacTables make_mac_tables(Ctx& C, const GmacBuild& b, const std::vector<int64_t>& wcodes, int level,
                                 bool single, bool pq, int na, std::vector<void*>& owner) {
  const int nout = (int)b.goff.size() - 1;
  // signature of an output: per group, whether it has a plaintext, and its inputs
  std::map<std::vector<int>, int> open;   // signature -> last class with it
  std::vector<std::vector<int>> members;
  for (int o = 0; o < nout; o++) {
    std::vector<int> sig;
    for (int g = b.goff[o]; g < b.goff[o + 1]; g++) {
      sig.push_back(b.mask[g] ? -2 : -1);
      for (int k = b.toff[g]; k < b.toff[g + 1]; k++) sig.push_back(b.tin[k]);
    }
    int c = -1;
    if (!single) {
      auto it = open.find(sig);
      if (it != open.end() && (int)members[it->second].size() < fk::kMacOut) c = it->second;
    }
    if (c < 0) {
      c = (int)members.size();
      members.push_back({});
      if (!single) open[sig] = c;
    }
    members[c].push_back(o);
  }
  // classes ordered by row width (next power of two of the output count), one
  // launch per width
  auto width_of = [](int n) {
    int w = 1;
    while (w < n) w <<= 1;
    return w;
  };
  // plaintext form of a class: none, the same plaintext for every member in
  // each group, or one per (group, member)
  auto ptm_of = [&](const std::vector<int>& mem) {
    bool any = false, shared = true;
    for (int gr = 0; gr < b.goff[mem[0] + 1] - b.goff[mem[0]]; gr++)
      for (int o : mem) {
        any = any || b.mask[b.goff[o] + gr];
        shared = shared && b.mask[b.goff[o] + gr] == b.mask[b.goff[mem[0]] + gr];
      }
    return !any ? (int)fk::kPtNone : shared ? (int)fk::kPtShared : (int)fk::kPtEach;
  };
  // diagonal class: every group one term of weight 1 and a plaintext for every member
  auto is_diag = [&](const std::vector<int>& mem) {
    for (int o : mem)
      for (int g = b.goff[o]; g < b.goff[o + 1]; g++) {
        if (!b.mask[g] || b.toff[g + 1] - b.toff[g] != 1) return false;
        const int k = b.toff[g];
        if (pq && b.tin[k] < na) return false;   // A terms carry the factor P
        if (b.tw[k] >= 0 && wcodes[b.tw[k]] != 1) return false;
      }
    return true;
  };
  const int64_t fast_lim = 1LL << fk::kFastWBits;
  auto is_fast = [&](const std::vector<int>& mem) {
    for (int o : mem)
      for (int k = b.toff[b.goff[o]]; k < b.toff[b.goff[o + 1]]; k++) {
        if (pq && b.tin[k] < na) return false;   // A terms carry the factor P
        const int w = b.tw[k];
        if (w >= 0 && !(wcodes[w] > -fast_lim && wcodes[w] < fast_lim)) return false;
      }
    return true;
  };
  auto chunk_of = [&](const std::vector<int>& m) {
    const int ng = b.goff[m[0] + 1] - b.goff[m[0]];
    const int nt = b.toff[b.goff[m[0] + 1]] - b.toff[b.goff[m[0]]];
    return nt >= 6 * ng ? fk::kMacChunk : 4;
  };
  // single-term class: every group one term, one plaintext per group shared
  // by the class (or none) -- two modular products per term beat the exact
  // split-and-accumulate of the general form
  auto is_one = [&](const std::vector<int>& mem) {
    if (is_diag(mem) || ptm_of(mem) != fk::kPtShared) return false;
    for (int o : mem)
      for (int g = b.goff[o]; g < b.goff[o + 1]; g++)
        if (b.toff[g + 1] - b.toff[g] != 1) return false;
    return true;
  };
  auto seg_key = [&](const std::vector<int>& m) {
    const bool dg = is_diag(m), one = is_one(m);
    return std::make_tuple(width_of((int)m.size()), dg ? (int)fk::kPtEach : ptm_of(m), (int)dg, (int)one,
                           (int)(!dg && !one && is_fast(m)), chunk_of(m));
  };
  {   // classes with a plaintext per (group, output) hold at most kMacOutEach outputs
    std::vector<std::vector<int>> split;
    for (auto& mem : members) {
      if ((int)mem.size() <= fk::kMacOutEach || is_diag(mem) || ptm_of(mem) != fk::kPtEach) {
        split.push_back(mem);
        continue;
      }
      for (size_t o = 0; o < mem.size(); o += fk::kMacOutEach)
        split.push_back(std::vector<int>(mem.begin() + o, mem.begin() + std::min(mem.size(), o + fk::kMacOutEach)));
    }
    members.swap(split);
  }
  std::stable_sort(members.begin(), members.end(), [&](const std::vector<int>& x, const std::vector<int>& y) {
    return seg_key(x) < seg_key(y);
  });
  constexpr int kZero = INT32_MIN;   // padding weight 0
  std::vector<fk::MacClass> cls;
  std::vector<int> cls_out, toff{0}, tin, wi;   // wi: weight index per (class term, row slot), -1: weight 1
  std::vector<char> wa;                         // the term reads an A input
  std::vector<char> wfast;                      // the entry belongs to a fast class (signed code stored)
  std::vector<const uint64_t*> mask;
  MacTables T;
  int ngroups = 0;
  for (auto& mem : members) {
    const int rep = mem[0], no = (int)mem.size(), W = width_of(no);
    const bool diag = is_diag(mem), one = is_one(mem), fast = !diag && !one && is_fast(mem);
    const int ptm = diag ? (int)fk::kPtEach : ptm_of(mem), chunk = chunk_of(mem);
    if (T.seg.empty() || T.seg.back().width != W || T.seg.back().ptm != ptm || T.seg.back().diag != diag ||
        T.seg.back().one != one || T.seg.back().fast != fast || T.seg.back().chunk != chunk)
      T.seg.push_back(MacSeg{(int)cls.size(), 0, W, ptm, diag, one, fast, chunk, 0.0, 0.0});
    for (int r = 0; r < b.toff[b.goff[rep + 1]] - b.toff[b.goff[rep]]; r++)
      for (int o = 0; o < W; o++) wfast.push_back(fast);
    MacSeg& sg = T.seg.back();
    sg.n++;
    fk::MacClass K;
    K.g0 = ngroups;
    K.ng = b.goff[rep + 1] - b.goff[rep];
    K.o0 = (int)cls_out.size();
    K.nout = no;
    K.w0 = (int)wi.size();
    K.m0 = (int)mask.size();
    for (int o : mem) cls_out.push_back(o);
    sg.words += 2.0 * no;   // outputs written
    for (int gr = 0; gr < K.ng; gr++) {
      const int g = b.goff[rep] + gr;
      for (int k = b.toff[g]; k < b.toff[g + 1]; k++) {
        tin.push_back(b.tin[k]);
        sg.words += 2.0;   // input read (both polys)
      }
      if (!diag) sg.mm += 2.0 * no * (b.toff[g + 1] - b.toff[g]);   // a weight product per term and output
      toff.push_back((int)tin.size());
      ngroups++;
      const uint64_t* prev = nullptr;
      for (int o = 0; o < W; o++) {
        const uint64_t* m = o < no ? b.mask[b.goff[mem[o]] + gr] : nullptr;
        mask.push_back(m);
        if (m && m != prev) sg.words += 1.0;   // plaintext read (one poly)
        if (m) sg.mm += 2.0;                    // a plaintext product per (group, output)
        if (m) prev = m;
      }
    }
    // weights term-major, row-slot-minor
    const int nterm = b.toff[b.goff[rep + 1]] - b.toff[b.goff[rep]];
    for (int r = 0; r < nterm; r++)
      for (int o = 0; o < W; o++) {
        wi.push_back(o < no ? b.tw[b.toff[b.goff[mem[o]]] + r] : kZero);
        wa.push_back(b.tin[b.toff[b.goff[rep]] + r] < na);
      }
    cls.push_back(K);
  }
  T.n = (int)cls.size();
  tin.resize(tin.size() + fk::kMacChunk, 0);   // whole chunks of indices are read at once
  T.cls = upload(C, cls, owner);
  T.cls_out = upload(C, cls_out, owner);
  T.mask = (const uint64_t**)upload(C, mask, owner);
  T.toff = upload(C, toff, owner);
  T.tin = upload(C, tin, owner);
  // weight residues per limb; in the extended basis the A inputs (Q only)
  // enter as P x: weight * P on the Q limbs, zero on the P limbs
  const int nq = level + 1, nlimbs = pq ? nq + C.K : nq;
  const LevelTabs& LT = level_tabs(C, level);
  T.ews = std::max<long long>(1, (long long)wi.size());
  std::vector<d2> ew((size_t)nlimbs * T.ews, d2{0, 0});
  for (int l = 0; l < nlimbs; l++) {
    const uint64_t q = C.primes[pq ? LT.h_eprime[l] : l];
    for (size_t k = 0; k < wi.size(); k++) {
      if (wfast[k]) {   // the signed code itself
        const int64_t code = wi[k] == kZero ? 0 : wi[k] < 0 ? 1 : wcodes[wi[k]];
        ew[(size_t)l * T.ews + k] = d2{(double)code, 0.0};
        continue;
      }
      const int64_t v = wi[k] == kZero ? 0 : wi[k] < 0 ? 1 : wcodes[wi[k]] % (int64_t)q;
      uint64_t r = (uint64_t)(v < 0 ? v + (int64_t)q : v);
      if (pq && wa[k]) r = l < nq ? mulmod(r, LT.h_pmod[l], q) : 0;
      ew[(size_t)l * T.ews + k] = cpair(r, q);
    }
  }
  T.ew = upload(C, ew, owner);
  std::vector<double> wc(T.ews, 0.0);
  for (size_t k = 0; k < wi.size(); k++)
    if (wfast[k]) wc[k] = (double)(wi[k] == kZero ? 0 : wi[k] < 0 ? 1 : wcodes[wi[k]]);
  T.wc = upload(C, wc, owner);
  return T;
}

GmacStage make_gmac(Ctx& C, const GmacBuild& b, const std::vector<int64_t>& wcodes, int level,
                    std::vector<void*>& owner, bool pq, int na) {
  GmacStage g;
  g.n_out = (int)b.goff.size() - 1;
  g.n_terms = (long long)b.tin.size();
  g.pq = pq;
  if (pq) g.eprime = level_tabs(C, level).eprime;
  for (auto* m : b.mask) g.n_masked += m != nullptr;
  if (g.n_out > 0) {
    g.batched = make_mac_tables(C, b, wcodes, level, false, pq, na, owner);
    g.single = make_mac_tables(C, b, wcodes, level, true, pq, na, owner);
  }
  return g;
}

u64* encode_plaintexts(Ctx& C, const std::vector<std::vector<double>>& slots, double scale, int level,
                       std::vector<void*>& owner, bool ext) {
  const LevelTabs& LT = level_tabs(C, level);
  const int N = C.N, nl = ext ? level + 1 + C.K : level + 1, n = (int)slots.size();
  std::vector<uint64_t> h((size_t)n * nl * N);
  const int nthr = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  for (int w = 0; w < nthr; w++)
    th.emplace_back([&, w] {
      std::vector<int64_t> m(N);
      for (int t = w; t < n; t += nthr) {
        fh::encode_real(C.logn, slots[t].data(), scale, m.data());
        for (int i = 0; i < nl; i++) {
          const int64_t q = (int64_t)C.primes[ext ? LT.h_eprime[i] : i];
          uint64_t* dst = &h[((size_t)t * nl + i) * N];
          for (int c = 0; c < N; c++) {
            int64_t v = m[c] % q;
            dst[c] = (uint64_t)(v < 0 ? v + q : v);
          }
        }
      }
    });
  for (auto& t : th) t.join();
  u64* d = upload(C, h, owner);
  fk::PrimeMap pm = identity_map(nl);
  if (ext)
    for (int i = 0; i < nl; i++) pm.p[i] = LT.h_eprime[i];
  ntt(C, false, d, d, (long long)nl * N, (long long)nl * N, n * nl, nl, pm, nullptr);
  fb::sync(nullptr);
  return d;
}

// Integer weight code: the binary64 product w * scale rounded half away from
// zero (above 2^53 the product is already an integer), |code| < 2^62.
int64_t weight_code(double w, double scale) {
  const double v = w * scale;
  if (!(std::fabs(v) < 4611686018427387904.0)) fail(FENC_EINVAL, "weight too large for its scale");
  return (int64_t)std::round(v);
}

void split_scale(double T, double& dw, double& dm) {
  int e = 0;
  std::frexp(T, &e);
  dw = std::ldexp(1.0, (e - 2) >> 1);   // 2^floor((e-2)/2): codes of |w| < 0.5 below 2^23 for T < 2^52
  dm = T / dw;
}

}  // namespace fr

fenc_ctx::~fenc_ctx() {
  plans.clear();
  for (void* p : owned) fb::dev_free(p);
}
