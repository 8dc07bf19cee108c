// C entry points of the oracle for the Python test harness.  TEST INFRASTRUCTURE.
// Data crosses this boundary as plain arrays: ciphertext batches are
// [n_ct][2][level+1][N] uint64 residues in coefficient form.
#include <chrono>
#include <cmath>
#include <cstring>
#include <thread>
#include <stdexcept>
#include <string>
#include "orc_method.h"

using namespace orc;

static thread_local std::string g_err;

#define GUARD_BEGIN try {
#define GUARD_END(ret)                 \
  }                                    \
  catch (const std::exception& e) {    \
    g_err = e.what();                  \
    return ret;                        \
  }

struct OrcLayout {
  int kind, bs, c, h, w, M, S, m, bsg, cpc, nbg, ncg, rep, dil, level, d, nfeat;
  double scale;
  int* pos;   // caller buffer (nfeat entries) or null
};

struct Batch {
  Layout L;
  std::vector<Ct> cts;
};

static void to_c(const Layout& L, OrcLayout* o) {
  o->kind = L.kind; o->bs = L.bs; o->c = L.c; o->h = L.h; o->w = L.w; o->M = L.M; o->S = L.S;
  o->m = L.m; o->bsg = L.bsg; o->cpc = L.cpc; o->nbg = L.nbg; o->ncg = L.ncg; o->rep = L.rep;
  o->dil = L.dil; o->level = L.level; o->d = L.d; o->nfeat = L.nfeat; o->scale = L.scale;
  if (o->pos && L.kind == KIND_VECTOR)
    for (int i = 0; i < L.nfeat; i++) o->pos[i] = L.pos[i];
}

static Layout from_c(const OrcLayout* o) {
  Layout L;
  L.kind = o->kind; L.bs = o->bs; L.c = o->c; L.h = o->h; L.w = o->w; L.M = o->M; L.S = o->S;
  L.m = o->m; L.bsg = o->bsg; L.cpc = o->cpc; L.nbg = o->nbg; L.ncg = o->ncg; L.rep = o->rep;
  L.dil = o->dil; L.level = o->level; L.d = o->d; L.nfeat = o->nfeat; L.scale = o->scale;
  if (L.kind == KIND_VECTOR) L.pos.assign(o->pos, o->pos + o->nfeat);
  return L;
}

static RPoly poly_from(const Context& C, const uint64_t* p, int nlimb, const std::vector<int>& pidx) {
  RPoly r = poly_zero(C, pidx);
  for (int l = 0; l < nlimb; l++) std::memcpy(r.c[l].data(), p + (size_t)l * C.N, C.N * 8);
  return r;
}

static void poly_to(const Context& C, const RPoly& r, uint64_t* p) {
  for (size_t l = 0; l < r.c.size(); l++) std::memcpy(p + l * C.N, r.c[l].data(), C.N * 8);
}

static Ct ct_from(const Context& C, const uint64_t* p, int level, double scale) {
  Ct ct;
  const size_t limb = (size_t)(level + 1) * C.N;
  ct.c0 = poly_from(C, p, level + 1, q_basis(level));
  ct.c1 = poly_from(C, p + limb, level + 1, q_basis(level));
  ct.level = level;
  ct.scale = scale;
  return ct;
}

static void ct_to(const Context& C, const Ct& ct, uint64_t* p) {
  const size_t limb = (size_t)(ct.level + 1) * C.N;
  poly_to(C, ct.c0, p);
  poly_to(C, ct.c1, p + limb);
}

static void counts_to(const Counts& c, long* o) {
  if (!o) return;
  long v[10] = {c.inner_rot, c.outer_rot, c.other_rot, c.ks, c.modup, c.moddown,
                c.pmult, c.smult, c.rescale, c.relin};
  for (int i = 0; i < 10; i++) o[i] = v[i];
}

extern "C" {

const char* orc_last_error() { return g_err.c_str(); }

void* orc_new(int logN, int nq, int qbits, int np, int pbits, int dnum, double log2scale,
              uint64_t seed) {
  GUARD_BEGIN
  Params p;
  p.logN = logN; p.nq = nq; p.qbits = qbits; p.np = np; p.pbits = pbits; p.dnum = dnum;
  p.log2scale = log2scale; p.seed = seed;
  return new Context(p);
  GUARD_END(nullptr)
}

void orc_free(void* c) { delete (Context*)c; }

int orc_primes(void* c, uint64_t* out) {
  Context* C = (Context*)c;
  for (size_t i = 0; i < C->primes.size(); i++) out[i] = C->primes[i];
  return (int)C->primes.size();
}

void orc_psi(void* c, uint64_t* out) {
  Context* C = (Context*)c;
  for (size_t i = 0; i < C->ring.size(); i++) out[i] = C->ring[i].psi;
}

void orc_secret(void* c, int64_t* out) {
  Context* C = (Context*)c;
  for (int i = 0; i < C->N; i++) out[i] = C->s[i];
}

int orc_is_prime(uint64_t n) { return is_prime(n) ? 1 : 0; }
uint64_t orc_rng(uint64_t seed, uint64_t tag, uint64_t i) { return rng(seed, tag, i); }
int orc_ternary(uint64_t seed, uint64_t tag, uint64_t i) { return sample_ternary(seed, tag, i); }
int orc_gauss(uint64_t seed, uint64_t tag, uint64_t i) { return sample_gauss(seed, tag, i); }
uint64_t orc_uniform(uint64_t seed, uint64_t tag, uint64_t i, uint64_t q) { return sample_uniform(seed, tag, i, q); }
void orc_gauss_cdt(uint64_t* out) {
  const std::vector<u64>& T = gauss_cdt();
  for (size_t i = 0; i < T.size(); i++) out[i] = T[i];
}

int orc_polymul(void* c, int pidx, const uint64_t* a, const uint64_t* b, uint64_t* out, int schoolbook) {
  GUARD_BEGIN
  Context* C = (Context*)c;
  RPoly A = poly_from(*C, a, 1, {pidx}), B = poly_from(*C, b, 1, {pidx});
  RPoly R = schoolbook ? poly_mul_schoolbook(*C, A, B) : poly_mul(*C, A, B);
  poly_to(*C, R, out);
  return 0;
  GUARD_END(-1)
}

int orc_ntt(void* c, int pidx, uint64_t* a, int inverse) {
  GUARD_BEGIN
  Context* C = (Context*)c;
  Vec v(a, a + C->N);
  if (inverse) C->ring[pidx].intt(v); else C->ring[pidx].ntt(v);
  std::memcpy(a, v.data(), C->N * 8);
  return 0;
  GUARD_END(-1)
}

int orc_automorph(void* c, int pidx, const uint64_t* a, uint64_t g, uint64_t* out) {
  GUARD_BEGIN
  Context* C = (Context*)c;
  poly_to(*C, automorph(*C, poly_from(*C, a, 1, {pidx}), g), out);
  return 0;
  GUARD_END(-1)
}

uint64_t orc_galois(void* c, int64_t shift) { return ((Context*)c)->galois(shift); }

int orc_encode_int(void* c, const double* re, const double* im, double scale, int64_t* out, int direct) {
  GUARD_BEGIN
  Context* C = (Context*)c;
  std::vector<double> R(re, re + C->ns), I;
  if (im) I.assign(im, im + C->ns);
  std::vector<i64> m = direct ? encode_int_direct(*C, R, I, scale) : encode_int(*C, R, I, scale);
  for (int i = 0; i < C->N; i++) out[i] = m[i];
  return 0;
  GUARD_END(-1)
}

int orc_encode(void* c, const double* re, const double* im, double scale, int level, uint64_t* out) {
  GUARD_BEGIN
  Context* C = (Context*)c;
  std::vector<double> R(re, re + C->ns), I;
  if (im) I.assign(im, im + C->ns);
  poly_to(*C, encode(*C, R, I, scale, q_basis(level)), out);
  return 0;
  GUARD_END(-1)
}

int orc_decode(void* c, const uint64_t* limb0, double scale, double* re, double* im) {
  GUARD_BEGIN
  Context* C = (Context*)c;
  std::vector<double> R, I;
  decode(*C, Vec(limb0, limb0 + C->N), C->primes[0], scale, R, I);
  for (int j = 0; j < C->ns; j++) { re[j] = R[j]; if (im) im[j] = I[j]; }
  return 0;
  GUARD_END(-1)
}

int orc_encrypt(void* c, const uint64_t* pt, int level, double scale, uint64_t seed, uint64_t ct_index,
                uint64_t* out) {
  GUARD_BEGIN
  Context* C = (Context*)c;
  ct_to(*C, encrypt(*C, poly_from(*C, pt, level + 1, q_basis(level)), level, scale, seed, ct_index), out);
  return 0;
  GUARD_END(-1)
}

int orc_decrypt(void* c, const uint64_t* ct, int level, uint64_t* out) {
  GUARD_BEGIN
  Context* C = (Context*)c;
  poly_to(*C, decrypt(*C, ct_from(*C, ct, level, 1.0)), out);
  return 0;
  GUARD_END(-1)
}

int orc_switch_key(void* c, uint64_t keyid, uint64_t* out) {
  GUARD_BEGIN
  Context* C = (Context*)c;
  std::vector<std::vector<RPoly>> k = gen_switch_key(*C, keyid);
  const size_t per = (size_t)C->np_total() * C->N;
  for (size_t j = 0; j < k.size(); j++)
    for (int t = 0; t < 2; t++) poly_to(*C, k[j][t], out + (j * 2 + t) * per);
  return (int)k.size();
  GUARD_END(-1)
}

int orc_mod_up(void* c, const uint64_t* d, int level, uint64_t* out) {
  GUARD_BEGIN
  Context* C = (Context*)c;
  std::vector<RPoly> e = mod_up(*C, poly_from(*C, d, level + 1, q_basis(level)), level);
  const size_t per = (size_t)(level + 1 + C->K) * C->N;
  for (size_t j = 0; j < e.size(); j++) poly_to(*C, e[j], out + j * per);
  return (int)e.size();
  GUARD_END(-1)
}

int orc_mod_down_rescale(void* c, const uint64_t* a, int level, uint64_t* out) {
  GUARD_BEGIN
  Context* C = (Context*)c;
  poly_to(*C, mod_down_rescale(*C, poly_from(*C, a, level + 1 + C->K, qp_basis(*C, level)), level), out);
  return 0;
  GUARD_END(-1)
}

int orc_mod_down(void* c, const uint64_t* a, int level, uint64_t* out) {
  GUARD_BEGIN
  Context* C = (Context*)c;
  poly_to(*C, mod_down(*C, poly_from(*C, a, level + 1 + C->K, qp_basis(*C, level)), level), out);
  return 0;
  GUARD_END(-1)
}

int orc_rotate(void* c, const uint64_t* ct, int level, const int64_t* shifts, int n, uint64_t* out) {
  GUARD_BEGIN
  Context* C = (Context*)c;
  std::vector<i64> sh(shifts, shifts + n);
  std::vector<Ct> r = rotate_hoisted(*C, ct_from(*C, ct, level, 1.0), sh);
  const size_t per = 2 * (size_t)(level + 1) * C->N;
  for (int i = 0; i < n; i++) ct_to(*C, r[i], out + i * per);
  return 0;
  GUARD_END(-1)
}

// the extended-basis forms moved down: mode 0 rotations (ModDown of
// rotate_hoisted_pq), mode 1 the lift P x (ModDown of lift_pq, shifts unused)
int orc_pq_roundtrip(void* c, const uint64_t* ct, int level, const int64_t* shifts, int n, int mode, uint64_t* out) {
  GUARD_BEGIN
  Context* C = (Context*)c;
  const Ct x = ct_from(*C, ct, level, 1.0);
  const size_t per = 2 * (size_t)(level + 1) * C->N;
  if (mode == 1) {
    ct_to(*C, mod_down_ct(*C, lift_pq(*C, x)), out);
    return 0;
  }
  std::vector<Ct> r = rotate_hoisted_pq(*C, x, std::vector<i64>(shifts, shifts + n));
  for (int i = 0; i < n; i++) ct_to(*C, mod_down_ct(*C, r[i]), out + i * per);
  return 0;
  GUARD_END(-1)
}

int orc_rotate_sum(void* c, const uint64_t* z0, const uint64_t* zs, const int64_t* shifts, int n,
                   int level, uint64_t* out) {
  GUARD_BEGIN
  Context* C = (Context*)c;
  const size_t per = 2 * (size_t)(level + 1) * C->N;
  Ct a;
  if (z0) a = ct_from(*C, z0, level, 1.0);
  std::vector<Ct> v;
  for (int i = 0; i < n; i++) v.push_back(ct_from(*C, zs + i * per, level, 1.0));
  std::vector<const Ct*> p;
  for (auto& x : v) p.push_back(&x);
  ct_to(*C, rotate_sum_lazy(*C, z0 ? &a : nullptr, p, std::vector<i64>(shifts, shifts + n)), out);
  return 0;
  GUARD_END(-1)
}

int orc_rescale(void* c, const uint64_t* ct, int level, uint64_t* out) {
  GUARD_BEGIN
  Context* C = (Context*)c;
  ct_to(*C, rescale(*C, ct_from(*C, ct, level, 1.0)), out);
  return 0;
  GUARD_END(-1)
}

int orc_square_relin(void* c, const uint64_t* ct, int level, uint64_t* out) {
  GUARD_BEGIN
  Context* C = (Context*)c;
  ct_to(*C, square_relin(*C, ct_from(*C, ct, level, 1.0), 1), out);
  return 0;
  GUARD_END(-1)
}

// ----------------------------------------------------------------- method
double orc_rot_total_formula(double BS, double Nin, double Nout, double K, double S, double alpha) {
  return rot_total_formula(BS, Nin, Nout, K, S, alpha);
}
double orc_rot_inner_formula_eq(double Nin, double K, double S, double M, double alpha) {
  return rot_inner_formula_eq(Nin, K, S, M, alpha);
}
double orc_optimal_S(double K, double Nin, double Nout, double alpha, double BS) {
  return optimal_S_closed_form(K, Nin, Nout, alpha, BS);
}

int orc_plan_layout(void* c, int bs, int ch, int h, int w, int k, int cout, int s_override, OrcLayout* out) {
  GUARD_BEGIN
  to_c(plan_layout(*(Context*)c, bs, ch, h, w, k, cout, s_override), out);
  return 0;
  GUARD_END(-1)
}

int orc_fragment_layout(void* c, int bs, int ch, int h, int w, int S, OrcLayout* out) {
  GUARD_BEGIN
  to_c(fragment_layout(*(Context*)c, bs, ch, h, w, S), out);
  return 0;
  GUARD_END(-1)
}

int orc_token_layout(void* c, int n, int E, int S, OrcLayout* out) {
  GUARD_BEGIN
  to_c(token_layout(*(Context*)c, n, E, S), out);
  return 0;
  GUARD_END(-1)
}

int orc_element_slots(const OrcLayout* lay, int b, int ch, int hh, int ww, int* out, int cap) {
  GUARD_BEGIN
  Layout L = from_c(lay);
  std::vector<std::pair<int, int>> sl;
  element_slots(L, b, ch, hh, ww, sl);
  int n = 0;
  for (auto& p : sl)
    if (n < cap) { out[2 * n] = p.first; out[2 * n + 1] = p.second; n++; }
  return n;
  GUARD_END(-1)
}

void* orc_encrypt_tensor(void* c, const OrcLayout* lay, const double* x, uint64_t seed) {
  GUARD_BEGIN
  Context* C = (Context*)c;
  Batch* b = new Batch;
  b->L = from_c(lay);
  b->cts = encrypt_batch(*C, b->L, encode_fragment(*C, b->L, x), seed);
  return b;
  GUARD_END(nullptr)
}

int orc_encode_tensor(void* c, const OrcLayout* lay, const double* x, uint64_t* out) {
  GUARD_BEGIN
  Context* C = (Context*)c;
  Layout L = from_c(lay);
  std::vector<RPoly> pts = encode_fragment(*C, L, x);
  const size_t per = (size_t)(L.level + 1) * C->N;
  for (size_t t = 0; t < pts.size(); t++) poly_to(*C, pts[t], out + t * per);
  return 0;
  GUARD_END(-1)
}

void* orc_batch_from(void* c, const OrcLayout* lay, const uint64_t* data) {
  GUARD_BEGIN
  Context* C = (Context*)c;
  Batch* b = new Batch;
  b->L = from_c(lay);
  const size_t per = 2 * (size_t)(b->L.level + 1) * C->N;
  for (int t = 0; t < b->L.n_ct(); t++) b->cts.push_back(ct_from(*C, data + t * per, b->L.level, b->L.scale));
  return b;
  GUARD_END(nullptr)
}

void orc_batch_free(void* b) { delete (Batch*)b; }

void orc_batch_layout(void* b, OrcLayout* out) { to_c(((Batch*)b)->L, out); }

int orc_batch_data(void* c, void* bp, uint64_t* out) {
  Context* C = (Context*)c;
  Batch* b = (Batch*)bp;
  const size_t per = 2 * (size_t)(b->L.level + 1) * C->N;
  for (size_t t = 0; t < b->cts.size(); t++) ct_to(*C, b->cts[t], out + t * per);
  return (int)b->cts.size();
}

int orc_decrypt_tensor(void* c, void* bp, double* x) {
  GUARD_BEGIN
  Batch* b = (Batch*)bp;
  decrypt_decode(*(Context*)c, b->L, b->cts, x);
  return 0;
  GUARD_END(-1)
}

// outs/n_outs: compute only those output ciphertexts (n_outs = 0: all); the
// batch then holds them in that order (its layout is the full output's)
void* orc_conv2d(void* c, void* bp, const double* w, int cout, int k, int stride, int pad, int groups,
                 long long pt_budget, int hoist, const OrcLayout* target, const double* bias, const int* outs,
                 int n_outs, int baby, long* counts) {
  GUARD_BEGIN
  Batch* in = (Batch*)bp;
  Batch* out = new Batch;
  Counts cnt;
  Layout T;
  if (target) T = from_c(target);
  std::vector<int> only(outs, outs + (n_outs > 0 ? n_outs : 0));
  out->cts = conv2d(*(Context*)c, in->L, in->cts, w, cout, k, stride, pad, groups, out->L, cnt, pt_budget, hoist,
                    target ? &T : nullptr, bias, n_outs > 0 ? &only : nullptr, baby);
  counts_to(cnt, counts);
  return out;
  GUARD_END(nullptr)
}

void* orc_avgpool2(void* c, void* bp, int hoist, long* counts) {
  GUARD_BEGIN
  Batch* in = (Batch*)bp;
  Batch* out = new Batch;
  Counts cnt;
  out->cts = avgpool2(*(Context*)c, in->L, in->cts, out->L, cnt, hoist);
  counts_to(cnt, counts);
  return out;
  GUARD_END(nullptr)
}

void* orc_square(void* c, void* bp, long* counts) {
  GUARD_BEGIN
  Batch* in = (Batch*)bp;
  Batch* out = new Batch;
  Counts cnt;
  out->cts = square_act(*(Context*)c, in->L, in->cts, out->L, cnt);
  counts_to(cnt, counts);
  return out;
  GUARD_END(nullptr)
}

void* orc_poly_act(void* c, void* bp, const double* coeffs, int n, long* counts) {
  GUARD_BEGIN
  Batch* in = (Batch*)bp;
  Batch* out = new Batch;
  Counts cnt;
  out->cts = poly_act(*(Context*)c, in->L, in->cts, std::vector<double>(coeffs, coeffs + n), out->L, cnt);
  counts_to(cnt, counts);
  return out;
  GUARD_END(nullptr)
}

void* orc_compress(void* c, void* bp, const OrcLayout* target, int hoist, long* counts) {
  GUARD_BEGIN
  Batch* in = (Batch*)bp;
  Batch* out = new Batch;
  Counts cnt;
  if (target) out->cts = compress_to(*(Context*)c, in->L, in->cts, from_c(target), out->L, cnt, hoist);
  else out->cts = compress(*(Context*)c, in->L, in->cts, out->L, cnt, hoist);
  counts_to(cnt, counts);
  return out;
  GUARD_END(nullptr)
}

void* orc_fc(void* c, void* bp, const double* w, int dout, const double* bias, const int* outs, int n_outs,
             long* counts) {
  GUARD_BEGIN
  Batch* in = (Batch*)bp;
  Batch* out = new Batch;
  Counts cnt;
  std::vector<int> only(outs, outs + (n_outs > 0 ? n_outs : 0));
  out->cts = fc(*(Context*)c, in->L, in->cts, w, dout, out->L, cnt, bias, n_outs > 0 ? &only : nullptr);
  counts_to(cnt, counts);
  return out;
  GUARD_END(nullptr)
}

// Wall time per operation of the oracle's primitives at `level`, each thread
// working on its own ciphertext (keys generated before the clock starts):
// out = [ModUp + one rotation (hoisted form, one shift), each further hoisted
// rotation, plaintext product, scalar product, rescale, square with
// relinearisation]; per-op time = wall time / (threads * reps).
int orc_time_ops(void* c, int level, int threads, int reps, double* out) {
  GUARD_BEGIN
  Context& C = *(Context*)c;
  if (level < 1 || level > C.L || threads < 1 || reps < 1) throw std::runtime_error("orc_time_ops: bad argument");
  gauss_cdt();
  C.key(C.galois(1));
  C.key(C.galois(2));
  C.key(0);
  const double scale = std::ldexp(1.0, (int)C.prm.log2scale);
  std::vector<Ct> cts;
  std::vector<double> z(C.ns);
  for (int t = 0; t < threads; t++) {
    for (int i = 0; i < C.ns; i++) z[i] = std::sin(0.1 * (i + t));
    cts.push_back(encrypt(C, encode(C, z, {}, scale, q_basis(level)), level, scale, 77, t));
  }
  const RPoly pt = encode(C, z, {}, scale, q_basis(level));
  auto wall = [&](auto op) {
    auto t0 = std::chrono::steady_clock::now();
    std::vector<std::thread> th;
    for (int t = 0; t < threads; t++)
      th.emplace_back([&, t] {
        orc_serial() = true;   // one operation per thread, none split further
        for (int r = 0; r < reps; r++) op(cts[t]);
      });
    for (auto& x : th) x.join();
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() / ((double)threads * reps);
  };
  const double r1 = wall([&](const Ct& x) { rotate_hoisted(C, x, {1}); });
  const double r2 = wall([&](const Ct& x) { rotate_hoisted(C, x, {1, 2}); });
  out[0] = r1;
  out[1] = r2 - r1;
  out[2] = wall([&](const Ct& x) { mul_plain(C, x, pt, scale); });
  out[3] = wall([&](const Ct& x) { mul_scalar(C, x, 12345, 1.0); });
  out[4] = wall([&](const Ct& x) { rescale(C, x); });
  out[5] = wall([&](const Ct& x) { square_relin(C, x, 1); });
  return 0;
  GUARD_END(-1)
}

int64_t orc_weight_code(double w, double scale) { return weight_code(w, scale); }
void orc_split_scale(double T, double* dw, double* dm) { split_scale(T, *dw, *dm); }

}  // extern "C"
