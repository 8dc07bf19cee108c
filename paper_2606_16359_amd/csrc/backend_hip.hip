// HIP backend: kernels for gfx950 and their launchers.
#include <hip/hip_runtime.h>
#include <mutex>
#include <stdexcept>
#include <string>

#define FENC_HD __host__ __device__
// device pass: table-held pointers are global memory (no generic/flat access)
#if defined(__HIP_DEVICE_COMPILE__)
#define FENC_GLOBAL __attribute__((address_space(1)))
#endif
#include "fenc_backend.h"

namespace {

// Execution interface for one GPU thread (see fenc_kernels.h).
struct GpuX {
  int bx, by, bz, nt;
  double* smem;
  template <class F>
  __device__ void phase(F f) {
    f((int)threadIdx.x);
    __syncthreads();
  }
};

__device__ inline GpuX here(double* smem) {
  GpuX x;
  x.bx = blockIdx.x;
  x.by = blockIdx.y;
  x.bz = blockIdx.z;
  x.nt = blockDim.x;
  x.smem = smem;
  return x;
}

void check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

void check_launch(const char* what) { check(hipGetLastError(), what); }

}  // namespace

#define FENC_KERNEL_LDS(NAME, ARGS)                                                   \
  __global__ void __launch_bounds__(256) k_##NAME(fk::ARGS a) {                        \
    extern __shared__ double smem[];                                                   \
    GpuX x = here(smem);                                                               \
    fk::NAME(x, a);                                                                    \
  }                                                                                    \
  void fb::NAME(Grid g, int threads, size_t lds, Stream s, const fk::ARGS& a) {        \
    hipLaunchKernelGGL(k_##NAME, dim3(g.x, g.y, g.z), dim3(threads), lds,              \
                       (hipStream_t)s, a);                                             \
    check_launch(#NAME);                                                               \
  }

// Kernels launched in the XCD-aware block order (1-D grid, coordinates decoded
// by xcd_coords).
#define FENC_KERNEL_XCD(NAME, ARGS)                                                   \
  __global__ void __launch_bounds__(256) k_##NAME(fk::ARGS a, unsigned gx, unsigned gy, unsigned gz) { \
    GpuX x = here(nullptr);                                                            \
    fk::xcd_coords(blockIdx.x, gx, gy, gz, x.bx, x.by, x.bz);                          \
    fk::NAME(x, a);                                                                    \
  }                                                                                    \
  void fb::NAME(Grid g, int threads, Stream s, const fk::ARGS& a) {                    \
    hipLaunchKernelGGL(k_##NAME, dim3(g.x * g.y * g.z), dim3(threads), 0,              \
                       (hipStream_t)s, a, g.x, g.y, g.z);                              \
    check_launch(#NAME);                                                               \
  }

#define FENC_KERNEL(NAME, ARGS)                                                       \
  __global__ void __launch_bounds__(256) k_##NAME(fk::ARGS a) {                        \
    GpuX x = here(nullptr);                                                            \
    fk::NAME(x, a);                                                                    \
  }                                                                                    \
  void fb::NAME(Grid g, int threads, Stream s, const fk::ARGS& a) {                    \
    hipLaunchKernelGGL(k_##NAME, dim3(g.x, g.y, g.z), dim3(threads), 0,                \
                       (hipStream_t)s, a);                                             \
    check_launch(#NAME);                                                               \
  }

FENC_KERNEL_LDS(ntt_fwd_cols, NttArgs)
FENC_KERNEL_LDS(ntt_fwd_rows, NttArgs)
FENC_KERNEL_LDS(ntt_inv_rows, NttArgs)
FENC_KERNEL_LDS(ntt_inv_cols, NttArgs)
FENC_KERNEL_LDS(ntt_fwd_cols16, NttArgs)
FENC_KERNEL_LDS(ntt_fwd_rows16, NttArgs)
FENC_KERNEL_LDS(ntt_fwd_rows_md, NttMdArgs)
FENC_KERNEL_LDS(ntt_fwd_rows16_md, NttMdArgs)
FENC_KERNEL_LDS(ntt_fwd_rows_rs, NttRsArgs)
FENC_KERNEL_LDS(ntt_fwd_rows16_rs, NttRsArgs)
FENC_KERNEL_LDS(ntt_fwd_cols_lift, NttLiftArgs)
FENC_KERNEL_LDS(ntt_fwd_cols16_lift, NttLiftArgs)
FENC_KERNEL_LDS(ntt_inv_rows16, NttArgs)
FENC_KERNEL_LDS(ntt_inv_cols16, NttArgs)
FENC_KERNEL(modup_fbc, ModUpArgs)
FENC_KERNEL_XCD(kip, KipArgs)
FENC_KERNEL_XCD(kip_own, KipArgs)
FENC_KERNEL(moddown_fbc, ModDownArgs)
FENC_KERNEL(rs_prep, RsPrepArgs)
FENC_KERNEL_XCD(gmac, GmacArgs)
FENC_KERNEL_XCD(gmac_pt, GmacArgs)
FENC_KERNEL_XCD(gmac_fast, GmacArgs)
FENC_KERNEL_XCD(gmac_pt_fast, GmacArgs)
FENC_KERNEL_XCD(gmac_ptv, GmacArgs)
FENC_KERNEL_XCD(gmac_ptv_fast, GmacArgs)
FENC_KERNEL_XCD(gmac_diag, GmacArgs)
FENC_KERNEL_XCD(gmac_one, GmacArgs)
FENC_KERNEL(tensor_square, SquareArgs)
FENC_KERNEL(lift_pq, LiftPqArgs)
FENC_KERNEL(lin_comb, LinArgs)
FENC_KERNEL(key_combine, KeyArgs)
FENC_KERNEL(enc_combine, EncArgs)
FENC_KERNEL(dec_combine, DecArgs)
FENC_KERNEL(small_to_rns, SmallArgs)
FENC_KERNEL(perm_rows, PermArgs)

namespace fb {

void* dev_alloc(size_t bytes) {
  void* p = nullptr;
  check(hipMalloc(&p, bytes ? bytes : 256), "hipMalloc");
  return p;
}

void dev_free(void* p) {
  if (p) (void)hipFree(p);
}

void device_sync() { check(hipDeviceSynchronize(), "hipDeviceSynchronize"); }

void h2d(void* dst, const void* src, size_t bytes) {
  if (bytes) check(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice), "hipMemcpy H2D");
}

void d2h(void* dst, const void* src, size_t bytes) {
  if (bytes) check(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost), "hipMemcpy D2H");
}

void d2d_async(void* dst, const void* src, size_t bytes, Stream s) {
  if (bytes) check(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, (hipStream_t)s), "hipMemcpyAsync D2D");
}

void sync(Stream s) { check(hipStreamSynchronize((hipStream_t)s), "hipStreamSynchronize"); }

bool capturing(Stream s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing((hipStream_t)s, &st) != hipSuccess) return false;
  return st == hipStreamCaptureStatusActive;
}

const char* backend_name() { return "hip-gfx950"; }

void* event_create() {
  hipEvent_t e;
  check(hipEventCreate(&e), "hipEventCreate");
  return (void*)e;
}
void event_record(void* e, Stream s) { check(hipEventRecord((hipEvent_t)e, (hipStream_t)s), "hipEventRecord"); }
float event_elapsed_ms(void* a, void* b) {
  check(hipEventSynchronize((hipEvent_t)b), "hipEventSynchronize");
  float ms = 0;
  check(hipEventElapsedTime(&ms, (hipEvent_t)a, (hipEvent_t)b), "hipEventElapsedTime");
  return ms;
}
void event_destroy(void* e) { (void)hipEventDestroy((hipEvent_t)e); }

int device_id() {
  int d = 0;
  check(hipGetDevice(&d), "hipGetDevice");
  return d;
}

}  // namespace fb

// Static device scratch of the no-allocation entry point: every GPU the
// library runs on holds one copy until the process ends.  Host code never
// uses the array's name as an address (on the host it is a stand-in): the
// device address comes from hipGetSymbolAddress, once per device, with that
// device current, and only that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[fb::kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

void* fb::scratch_base() {
  const int d = device_id();
  if (d < 0 || d >= kMaxDevices) throw std::runtime_error("scratch: device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[d]) {
    void* ptr = nullptr;
    check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[d] = ptr;
  }
  return g_scratch_ptr[d];
}
