// Sequential emulator of the device interface, for the CPU test suite only.
//
// It runs the same kernel bodies as the HIP backend (fenc_kernels.h): blocks
// are iterated (in parallel over OpenMP threads), threads of a block are
// iterated inside each barrier phase.  Device memory is host memory.  It lets
// the CPU tests check the kernels' index arithmetic and the host runtime
// against the oracle; the product library never contains it.
#include <cstdlib>
#include <cstring>
#include <stdexcept>
#include <vector>

#include "fenc_backend.h"

namespace {

struct CpuX {
  int bx, by, bz, nt;
  double* smem;
  template <class F>
  void phase(F f) {
    for (int t = 0; t < nt; t++) f(t);
  }
};

template <class F>
void run(fb::Grid g, int threads, size_t lds, F body, bool xcd = false) {
  const long long nb = (long long)g.x * g.y * g.z;
#pragma omp parallel
  {
    std::vector<double> sm(lds / 8 + 8);
#pragma omp for schedule(dynamic, 4)
    for (long long i = 0; i < nb; i++) {
      CpuX x;
      if (xcd) {
        fk::xcd_coords((unsigned)i, g.x, g.y, g.z, x.bx, x.by, x.bz);
      } else {
        x.bx = (int)(i % g.x);
        x.by = (int)((i / g.x) % g.y);
        x.bz = (int)(i / ((long long)g.x * g.y));
      }
      x.nt = threads;
      x.smem = sm.data();
      body(x);
    }
  }
}

}  // namespace

#define EMU_LDS(NAME, ARGS)                                                          \
  void fb::NAME(Grid g, int threads, size_t lds, Stream, const fk::ARGS& a) {         \
    run(g, threads, lds, [&](CpuX& x) { fk::NAME(x, a); });                           \
  }
#define EMU_XCD(NAME, ARGS)                                                          \
  void fb::NAME(Grid g, int threads, Stream, const fk::ARGS& a) {                     \
    run(g, threads, 0, [&](CpuX& x) { fk::NAME(x, a); }, true);                       \
  }
#define EMU(NAME, ARGS)                                                              \
  void fb::NAME(Grid g, int threads, Stream, const fk::ARGS& a) {                     \
    run(g, threads, 0, [&](CpuX& x) { fk::NAME(x, a); });                             \
  }

EMU_LDS(ntt_fwd_cols, NttArgs)
EMU_LDS(ntt_fwd_rows, NttArgs)
EMU_LDS(ntt_inv_rows, NttArgs)
EMU_LDS(ntt_inv_cols, NttArgs)
EMU_LDS(ntt_fwd_cols16, NttArgs)
EMU_LDS(ntt_fwd_rows16, NttArgs)
EMU_LDS(ntt_fwd_rows_md, NttMdArgs)
EMU_LDS(ntt_fwd_rows16_md, NttMdArgs)
EMU_LDS(ntt_fwd_rows_rs, NttRsArgs)
EMU_LDS(ntt_fwd_rows16_rs, NttRsArgs)
EMU_LDS(ntt_fwd_cols_lift, NttLiftArgs)
EMU_LDS(ntt_fwd_cols16_lift, NttLiftArgs)
EMU_LDS(ntt_inv_rows16, NttArgs)
EMU_LDS(ntt_inv_cols16, NttArgs)
EMU(modup_fbc, ModUpArgs)
EMU_XCD(kip, KipArgs)
EMU_XCD(kip_own, KipArgs)
EMU(moddown_fbc, ModDownArgs)
EMU(rs_prep, RsPrepArgs)
EMU_XCD(gmac, GmacArgs)
EMU_XCD(gmac_pt, GmacArgs)
EMU_XCD(gmac_fast, GmacArgs)
EMU_XCD(gmac_pt_fast, GmacArgs)
EMU_XCD(gmac_ptv, GmacArgs)
EMU_XCD(gmac_ptv_fast, GmacArgs)
EMU_XCD(gmac_diag, GmacArgs)
EMU_XCD(gmac_one, GmacArgs)
EMU(tensor_square, SquareArgs)
EMU(lift_pq, LiftPqArgs)
EMU(lin_comb, LinArgs)
EMU(key_combine, KeyArgs)
EMU(enc_combine, EncArgs)
EMU(dec_combine, DecArgs)
EMU(small_to_rns, SmallArgs)
EMU(perm_rows, PermArgs)

namespace fb {
// exact-size allocations, so that an address-sanitizer build of the emulator
// reports any read or write past the end of a buffer
void* dev_alloc(size_t bytes) {
  void* p = nullptr;
  if (posix_memalign(&p, 256, bytes ? bytes : 1) != 0 || !p) throw std::runtime_error("emulator: out of memory");
  std::memset(p, 0xA5, bytes);   // poison: kernels must not read unwritten memory
  return p;
}
void dev_free(void* p) { std::free(p); }
void device_sync() {}
void h2d(void* dst, const void* src, size_t bytes) { std::memcpy(dst, src, bytes); }
void d2h(void* dst, const void* src, size_t bytes) { std::memcpy(dst, src, bytes); }
void d2d_async(void* dst, const void* src, size_t bytes, Stream) { std::memcpy(dst, src, bytes); }
void sync(Stream) {}
bool capturing(Stream) { return false; }
const char* backend_name() { return "cpu-emulator"; }
void* event_create() { return nullptr; }
void event_record(void*, Stream) {}
float event_elapsed_ms(void*, void*) { return 0.f; }
void event_destroy(void*) {}
int device_id() { return 0; }
void* scratch_base() {
  static unsigned char* buf = [] {
    unsigned char* b = (unsigned char*)std::aligned_alloc(256, kScratchBytes);
    std::memset(b, 0xA5, kScratchBytes);
    return b;
  }();
  return buf;
}
}  // namespace fb
