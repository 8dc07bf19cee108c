// Device interface used by the host runtime: memory, streams and one launch
// function per kernel.  The product library implements it with HIP
// (backend_hip.hip); the host runtime itself contains no device code.
#pragma once
#include <cstddef>
#include "fenc_kernels.h"

namespace fb {

typedef void* Stream;   // hipStream_t

struct Grid {
  unsigned x, y, z;
};

void* dev_alloc(size_t bytes);                       // throws std::runtime_error
// Device address of the library's static scratch array on the current device
// (kScratchBytes, 256-byte aligned, shared by every call on that device); the
// first call on a device looks the address up, later calls return it.
constexpr size_t kScratchBytes = 64ull << 20;
void* scratch_base();
void dev_free(void* p);
void device_sync();                                  // waits for all work on the device
void h2d(void* dst, const void* src, size_t bytes);  // synchronous
void d2h(void* dst, const void* src, size_t bytes);  // synchronous (device-wide)
void d2d_async(void* dst, const void* src, size_t bytes, Stream s);
void sync(Stream s);
bool capturing(Stream s);
const char* backend_name();
int device_id();
// timing events on a stream (profiling of single kernels)
void* event_create();
void event_record(void* e, Stream s);
float event_elapsed_ms(void* start, void* stop);   // synchronises on stop
void event_destroy(void* e);

// NTT passes use fixed block shapes chosen by the runtime
void ntt_fwd_cols(Grid g, int threads, size_t smem, Stream s, const fk::NttArgs& a);
void ntt_fwd_rows(Grid g, int threads, size_t smem, Stream s, const fk::NttArgs& a);
void ntt_inv_rows(Grid g, int threads, size_t smem, Stream s, const fk::NttArgs& a);
void ntt_inv_cols(Grid g, int threads, size_t smem, Stream s, const fk::NttArgs& a);
// the same passes with radix-16 register rounds
void ntt_fwd_cols16(Grid g, int threads, size_t smem, Stream s, const fk::NttArgs& a);
void ntt_fwd_rows16(Grid g, int threads, size_t smem, Stream s, const fk::NttArgs& a);
void ntt_fwd_rows_md(Grid g, int threads, size_t smem, Stream s, const fk::NttMdArgs& a);
void ntt_fwd_rows16_md(Grid g, int threads, size_t smem, Stream s, const fk::NttMdArgs& a);
void ntt_fwd_rows_rs(Grid g, int threads, size_t smem, Stream s, const fk::NttRsArgs& a);
void ntt_fwd_cols_lift(Grid g, int threads, size_t smem, Stream s, const fk::NttLiftArgs& a);
void ntt_fwd_cols16_lift(Grid g, int threads, size_t smem, Stream s, const fk::NttLiftArgs& a);
void ntt_fwd_rows16_rs(Grid g, int threads, size_t smem, Stream s, const fk::NttRsArgs& a);
void ntt_inv_rows16(Grid g, int threads, size_t smem, Stream s, const fk::NttArgs& a);
void ntt_inv_cols16(Grid g, int threads, size_t smem, Stream s, const fk::NttArgs& a);
void modup_fbc(Grid g, int threads, Stream s, const fk::ModUpArgs& a);
void kip(Grid g, int threads, Stream s, const fk::KipArgs& a);
void kip_own(Grid g, int threads, Stream s, const fk::KipArgs& a);   // own limbs from the input
void moddown_fbc(Grid g, int threads, Stream s, const fk::ModDownArgs& a);
void rs_prep(Grid g, int threads, Stream s, const fk::RsPrepArgs& a);
void gmac(Grid g, int threads, Stream s, const fk::GmacArgs& a);
void gmac_pt(Grid g, int threads, Stream s, const fk::GmacArgs& a);
void gmac_fast(Grid g, int threads, Stream s, const fk::GmacArgs& a);
void gmac_pt_fast(Grid g, int threads, Stream s, const fk::GmacArgs& a);
void gmac_ptv(Grid g, int threads, Stream s, const fk::GmacArgs& a);
void gmac_ptv_fast(Grid g, int threads, Stream s, const fk::GmacArgs& a);
void gmac_diag(Grid g, int threads, Stream s, const fk::GmacArgs& a);
void gmac_one(Grid g, int threads, Stream s, const fk::GmacArgs& a);
void tensor_square(Grid g, int threads, Stream s, const fk::SquareArgs& a);
void lift_pq(Grid g, int threads, Stream s, const fk::LiftPqArgs& a);
void lin_comb(Grid g, int threads, Stream s, const fk::LinArgs& a);
void key_combine(Grid g, int threads, Stream s, const fk::KeyArgs& a);
void enc_combine(Grid g, int threads, Stream s, const fk::EncArgs& a);
void dec_combine(Grid g, int threads, Stream s, const fk::DecArgs& a);
void small_to_rns(Grid g, int threads, Stream s, const fk::SmallArgs& a);
void perm_rows(Grid g, int threads, Stream s, const fk::PermArgs& a);

}  // namespace fb
