// Plain CPU oracle for the FEnc^2 hot path (arXiv 2606.16359).
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
// includes this code; only the test suite, the smoke check and the CPU
// baseline leg of the benchmark load it.  It shares no code, header, table or
// constant generator with the HIP path.
//
// Every routine here is written for obviousness, not speed: modular products
// are `(unsigned __int128)a*b % q`, polynomials are kept in coefficient form
// between operations, automorphisms are applied by their coefficient-index
// definition, and the canonical-embedding encoder runs in __float128.
//
// Parity status of each function is listed in the header comment of the file
// that defines it.
#pragma once
#include <cstdint>
#include <string>
#include <vector>
#include <map>
#include <memory>
#include <mutex>
#include <algorithm>
#include <thread>
#include <exception>
#include <cstdlib>
#include <atomic>

namespace orc {

typedef uint64_t u64;
typedef int64_t i64;
typedef unsigned __int128 u128;
typedef __int128 i128;
typedef std::vector<u64> Vec;

// ---------------------------------------------------------------- modular ops
inline u64 addm(u64 a, u64 b, u64 q) { return (u64)(((u128)a + b) % q); }
inline u64 subm(u64 a, u64 b, u64 q) { return (u64)(((u128)a + q - b) % q); }
inline u64 mulm(u64 a, u64 b, u64 q) { return (u64)(((u128)a * b) % q); }
inline u64 negm(u64 a, u64 q) { return a == 0 ? 0 : q - a; }
u64 powm(u64 a, u64 e, u64 q);
u64 invm(u64 a, u64 q);                   // q prime, a != 0 mod q
inline u64 from_i64(i64 v, u64 q) {
  i128 r = (i128)v % (i128)q;
  if (r < 0) r += q;
  return (u64)r;
}
inline u64 from_i128(i128 v, u64 q) {
  i128 r = v % (i128)q;
  if (r < 0) r += q;
  return (u64)r;
}
bool is_prime(u64 n);                     // deterministic Miller-Rabin, 64-bit

// ---------------------------------------------------------------- sampler
// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) used as a keyed counter
// generator: output i of the SplitMix64 stream whose state starts at
// key(seed, tag).
u64 mix64(u64 z);
u64 rng(u64 seed, u64 tag, u64 i);
enum : u64 {
  TAG_SECRET = 1ull << 56,
  TAG_KEY_A = 2ull << 56,
  TAG_KEY_E = 3ull << 56,
  TAG_ENC_A = 4ull << 56,
  TAG_ENC_E = 5ull << 56,
};
inline u64 tag_key_a(u64 keyid, u64 digit, u64 prime) { return TAG_KEY_A | (keyid << 24) | (digit << 16) | prime; }
inline u64 tag_key_e(u64 keyid, u64 digit) { return TAG_KEY_E | (keyid << 24) | (digit << 16); }
inline u64 tag_enc_a(u64 ct, u64 prime) { return TAG_ENC_A | (ct << 16) | prime; }
inline u64 tag_enc_e(u64 ct) { return TAG_ENC_E | (ct << 16); }
int sample_ternary(u64 seed, u64 tag, u64 i);
int sample_gauss(u64 seed, u64 tag, u64 i);   // sigma 3.2, |e| <= 19
u64 sample_uniform(u64 seed, u64 tag, u64 i, u64 q);
const std::vector<u64>& gauss_cdt();           // 19 thresholds (63-bit)

// ---------------------------------------------------------------- ring
struct Params {
  int logN = 0, nq = 0, qbits = 0, np = 0, pbits = 0, dnum = 0;
  double log2scale = 0;
  u64 seed = 0;
};

struct Ring {
  int N = 0;
  u64 q = 0, psi = 0;                 // psi: primitive 2N-th root of unity
  Vec psi_pow, psi_inv_pow;           // psi^i, psi^-i  (i < N)
  Vec omega_pow, omega_inv_pow;       // (psi^2)^i      (i < N)
  u64 n_inv = 0;
  void init(int N_, u64 q_);
  // forward: A[j] = sum_i a_i psi^{(2j+1) i}   (natural order j)
  void ntt(Vec& a) const;
  void intt(Vec& a) const;
};
void cyclic_dft(Vec& a, const Vec& wpow, u64 q);   // in place, iterative radix 2

struct Context {
  Params prm;
  int N = 0, ns = 0, L = 0, K = 0, alpha = 0;   // L+1 = nq ; K = np ; alpha limbs per digit
  Vec primes;                                   // q_0..q_L, p_0..p_{K-1}
  std::vector<Ring> ring;
  std::vector<i64> s;                           // ternary secret coefficients
  // key cache: keyid -> [digit][2][prime][N] in NTT (evaluation) form
  struct KeySlot {
    std::once_flag once;
    std::vector<std::vector<std::vector<Vec>>> key;
  };
  std::map<u64, std::shared_ptr<KeySlot>> keys;
  std::shared_ptr<std::mutex> key_mu = std::make_shared<std::mutex>();   // guards the map `keys`
  explicit Context(const Params& p);
  int np_total() const { return L + 1 + K; }
  const std::vector<std::vector<std::vector<Vec>>>& key(u64 keyid);
  u64 galois(i64 shift) const;                  // 5^shift mod 2N
};

// prime search: the `count` largest primes below 2^bits with p = 1 mod 2N,
// skipping those already in `taken`
Vec find_primes(int bits, int logN, int count, const Vec& taken);
u64 find_psi(u64 q, int N);

// Threads for work over independent ciphertexts (ORC_THREADS, else the
// hardware's count, at most 16); the arithmetic of each item is unchanged.
// Set on a thread that must run par_for loops inline (the per-operation
// timings run one operation per thread).
inline bool& orc_serial() {
  static thread_local bool serial = false;
  return serial;
}

inline int orc_threads() {
  if (orc_serial()) return 1;
  const char* e = std::getenv("ORC_THREADS");
  int t = e ? std::atoi(e) : (int)std::thread::hardware_concurrency();
  return std::max(1, std::min(16, t));
}

// fn(i) for every i in [0, n), items spread over the threads
template <class F>
void par_for(int n, F fn) {
  const int T = std::min(n, orc_threads());
  if (T <= 1) {
    for (int i = 0; i < n; i++) fn(i);
    return;
  }
  std::atomic<int> next{0};
  std::exception_ptr err;
  std::mutex em;
  std::vector<std::thread> th;
  for (int t = 0; t < T; t++)
    th.emplace_back([&] {
      for (;;) {
        const int i = next++;
        if (i >= n) break;
        try {
          fn(i);
        } catch (...) {
          std::lock_guard<std::mutex> lock(em);
          if (!err) err = std::current_exception();
        }
      }
    });
  for (auto& x : th) x.join();
  if (err) std::rethrow_exception(err);
}


// ---------------------------------------------------------------- polys
// A polynomial in RNS form: limb l holds residues modulo primes[pidx[l]],
// coefficient form.
struct RPoly {
  std::vector<int> pidx;
  std::vector<Vec> c;
};
RPoly poly_zero(const Context& C, const std::vector<int>& pidx);
RPoly poly_mul(const Context& C, const RPoly& a, const RPoly& b);   // negacyclic, via NTT
RPoly poly_mul_schoolbook(const Context& C, const RPoly& a, const RPoly& b);
void poly_add_inplace(const Context& C, RPoly& a, const RPoly& b);
void poly_sub_inplace(const Context& C, RPoly& a, const RPoly& b);
RPoly poly_scalar(const Context& C, const RPoly& a, i64 s);
RPoly automorph(const Context& C, const RPoly& a, u64 g);           // X -> X^g
std::vector<int> q_basis(int level);                                 // 0..level
std::vector<int> qp_basis(const Context& C, int level);             // 0..level, L+1..L+K

// ---------------------------------------------------------------- ciphertext
struct Ct {
  RPoly c0, c1;
  int level = 0;
  double scale = 1.0;
};

// secret key operations
RPoly secret_poly(const Context& C, const std::vector<int>& pidx);
RPoly secret_square_poly(const Context& C, const std::vector<int>& pidx);
// key for target s' = sigma_g(s) (keyid = g) or s^2 (keyid = 0): coefficient form
// returns [digit][2][limb over qp basis at top level]
std::vector<std::vector<RPoly>> gen_switch_key(Context& C, u64 keyid);

Ct encrypt(const Context& C, const RPoly& pt, int level, double scale, u64 enc_seed, u64 ct_index);
RPoly decrypt(const Context& C, const Ct& ct);

// hybrid key switching pieces
std::vector<RPoly> mod_up(const Context& C, const RPoly& d, int level);   // beta extended digits
RPoly mod_down(const Context& C, const RPoly& a, int level);
// sum_j ext_j * key_j (poly 0 and 1), ext already automorphed
void key_inner_product(Context& C, const std::vector<RPoly>& ext, u64 keyid, int level,
                       RPoly& acc0, RPoly& acc1);

// rotations (left by `shift` slots), hoisted form: ModUp(c1) once, automorphism
// applied to the extended digits, one ModDown per output
std::vector<Ct> rotate_hoisted(Context& C, const Ct& x, const std::vector<i64>& shifts);
// hoisted rotations left in the extended basis Q_l U P (no ModDown):
// (KIP_0 + P sigma_g(c0), KIP_1); ModDown of the result is the rotated ciphertext
std::vector<Ct> rotate_hoisted_pq(Context& C, const Ct& x, const std::vector<i64>& shifts);
// (P x0, P x1) over Q_l U P (zero on the special primes); ModDown gives x back
Ct lift_pq(const Context& C, const Ct& x);
// ModDown of both polys of an extended-basis ciphertext
Ct mod_down_ct(const Context& C, const Ct& y);
// lazy form: y = z0 + sum_r Rot(z_r, shift_r) with a single ModDown
Ct rotate_sum_lazy(Context& C, const Ct* z0, const std::vector<const Ct*>& zs,
                   const std::vector<i64>& shifts);
Ct rescale(const Context& C, const Ct& x);
Ct add(const Context& C, const Ct& a, const Ct& b);
Ct mul_plain(const Context& C, const Ct& a, const RPoly& pt, double pt_scale);
Ct mul_scalar(const Context& C, const Ct& a, i64 s, double s_scale);
// k * a^2: tensor product scaled by the integer k, relinearised, no rescale
Ct square_relin(Context& C, const Ct& a, i64 k = 1);
// a * b: tensor product of two ciphertexts at one level, relinearised, no rescale
Ct mul_relin(Context& C, const Ct& a, const Ct& b);
// ModDown by P q_l of a polynomial over Q_l U P to Q_{l-1}: the special
// primes and q_l dropped by one fast base conversion
RPoly mod_down_rescale(const Context& C, const RPoly& a, int level);
// tensor product k (a x b): d0 = k a0 b0, d1 = k (a0 b1 + a1 b0), d2 = k a1 b1
void tensor(const Context& C, const Ct& a, const Ct& b, i64 k, RPoly& d0, RPoly& d1, RPoly& d2);
// (d.c0, d.c1) + KS(d2) relinearised and rescaled together: the key inner
// product of d2's extended digits plus P (d.c0, d.c1), ModDown by P q_l
Ct relin_rescale(Context& C, const Ct& d, const RPoly& d2);
// the same ciphertext at one level less (the last limb dropped)
Ct drop_last_limb(const Ct& a);
// base + k1 * x + k0 (k0 added to the constant coefficient of c0); base may be null
Ct lin_comb(const Context& C, const Ct* base, const Ct& x, i128 k1, i128 k0);

// ---------------------------------------------------------------- encoding
// m = round(scale * tau^{-1}(z)), complex slots z (ns entries), reduced mod primes
RPoly encode(const Context& C, const std::vector<double>& re, const std::vector<double>& im,
             double scale, const std::vector<int>& pidx);
std::vector<i64> encode_int(const Context& C, const std::vector<double>& re,
                            const std::vector<double>& im, double scale);
std::vector<i64> encode_int_direct(const Context& C, const std::vector<double>& re,
                                   const std::vector<double>& im, double scale);
// decode limb-0 residues (centered) divided by scale
void decode(const Context& C, const Vec& limb0, u64 q0, double scale,
            std::vector<double>& re, std::vector<double>& im);

}  // namespace orc
