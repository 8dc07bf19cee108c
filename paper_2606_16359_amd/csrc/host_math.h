// Host-side number theory, canonical-embedding codec and sampler of the
// library (parameter set-up and the client side of the protocol).
#pragma once
#include <cstdint>
#include <vector>

namespace fh {

typedef uint64_t u64;
typedef unsigned __int128 u128;

inline u64 mulmod(u64 a, u64 b, u64 q) { return (u64)((u128)a * b % q); }
u64 powmod(u64 a, u64 e, u64 q);
u64 invmod(u64 a, u64 q);
bool prime64(u64 n);
// the `count` largest primes p < 2^bits with p = 1 (mod 2N), excluding `skip`
std::vector<u64> ntt_primes(int bits, int logn, int count, const std::vector<u64>& skip);
// smallest generator-derived primitive 2N-th root: x = 2, 3, ... with (x^((p-1)/2N))^N = -1
u64 root_2n(u64 p, int logn);
unsigned bitrev(unsigned x, int bits);

// ---- sampler: SplitMix64 output stream, keyed by (seed, tag)
u64 splitmix_mix(u64 z);
u64 stream_word(u64 seed, u64 tag, u64 i);
int draw_ternary(u64 seed, u64 tag, u64 i);
int draw_gauss(u64 seed, u64 tag, u64 i);          // sigma 3.2, |e| <= 19
u64 draw_uniform(u64 seed, u64 tag, u64 i, u64 q);
const std::vector<u64>& gauss_thresholds();

namespace tag {
constexpr u64 secret = 1ull << 56;
inline u64 key_a(u64 id, u64 digit, u64 prime) { return (2ull << 56) | (id << 24) | (digit << 16) | prime; }
inline u64 key_e(u64 id, u64 digit) { return (3ull << 56) | (id << 24) | (digit << 16); }
inline u64 enc_a(u64 ct, u64 prime) { return (4ull << 56) | (ct << 16) | prime; }
inline u64 enc_e(u64 ct) { return (5ull << 56) | (ct << 16); }
}  // namespace tag

// ---- canonical embedding (double-double arithmetic)
// m_i = round_half_away(scale * tau^{-1}(z)_i), slots z (ns real values)
void encode_real(int logn, const double* z, double scale, int64_t* m);
// slots of a polynomial with small centred integer coefficients, divided by scale
void decode_real(int logn, const int64_t* m, double scale, double* z);

}  // namespace fh
