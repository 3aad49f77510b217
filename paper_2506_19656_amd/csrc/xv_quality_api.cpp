// xv_quality_api.cpp -- host side of the quality metrics reported beside
// PSNR: SSIM of the coded planes and the spectral angle of decoded cubes.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "xv_host.h"

using namespace xv;
using namespace xv::host;

extern "C" {

int xv_ssim(const xv_encoded* e, double* ssim, void* hip_stream) {
  if (!e || !ssim) return fail(XV_EINVAL, "null encoded cube or output");
  if (!e->frames || !e->recon)
    return fail(XV_EINVAL, "SSIM needs the converted frames and the reconstruction "
                           "(dropped by XV_FLAG_DROP_WORK; absent for a cube read from a bitstream)");
  const int bands = (int)e->bands;
  if (e->H < 11 || e->W < 11) {
    for (int b = 0; b < bands; b++) ssim[b] = NAN;
    return XV_OK;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  SsimArgs a;
  memset(&a, 0, sizeof a);
  a.frames = e->frames;
  a.recon = e->recon;
  double ws = 0.0;
  for (int i = 0; i < 11; i++) {
    const double d = (double)(i - 5);
    a.w[i] = exp(-(d * d) / (2.0 * 1.5 * 1.5));
    ws += a.w[i];
  }
  for (int i = 0; i < 11; i++) a.w[i] /= ws;
  const double L = (double)((1 << e->p.bit_depth) - 1);
  a.C1 = (0.01 * L) * (0.01 * L);
  a.C2 = (0.03 * L) * (0.03 * L);
  a.T = (int)e->T;
  a.Hp = e->Hp;
  a.Wp = e->Wp;
  a.H = (int)e->H;
  a.W = (int)e->W;
  a.bands = bands;
  ssim_tiles(a.H, a.W, &a.tiles_x, &a.tiles_y);
  const size_t nparts = (size_t)bands * a.T * a.tiles_x * a.tiles_y;
  void* mem = nullptr;
  hipError_t he = dev_alloc(&mem, (nparts + bands) * sizeof(double), s);
  if (he != hipSuccess) return fail(XV_ENOMEM, "SSIM scratch: %s", hipGetErrorString(he));
  a.part = (double*)mem;
  double* out = a.part + nparts;
  {
    ProfScope ps(XV_K_QUALITY, s, (double)e->T * e->H * e->W * bands * 4.0);
    he = launch_ssim(a, out, s);
  }
  if (he == hipSuccess) he = hipMemcpyAsync(ssim, out, bands * sizeof(double), hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  dev_free(mem, s);
  if (he != hipSuccess) return fail(XV_EHIP, "SSIM: %s", hipGetErrorString(he));
  return XV_OK;
}

}  // extern "C"

// The allocation-free spectral angle's scratch: per-block sums and counts
// of the largest grid of the per-block pass, then the two totals (65,552
// bytes).  Each GPU holds its own copy for the life of the process; host code
// reaches it only through the address hipGetSymbolAddress returns.
constexpr int kSaMaxBlocks = 4096;
constexpr size_t kSaScratchBytes = (size_t)kSaMaxBlocks * 16 + 16;
static __device__ __align__(256) unsigned char scratch[kSaScratchBytes];

namespace {

// Checks the two cubes and fills the kernel arguments; *nblocks receives the
// grid of the per-block pass (at most kSaMaxBlocks).

int sa_setup(const xv_cube* orig, const xv_cube* decoded, double* mean_rad, SaArgs* a,
             int* nblocks) {
  if (!mean_rad) return fail(XV_EINVAL, "null output");
  int rc = check_cube(orig, "original");
  if (rc != XV_OK) return rc;
  if ((rc = check_cube(decoded, "decoded")) != XV_OK) return rc;
  if (orig->T != decoded->T || orig->H != decoded->H || orig->W != decoded->W ||
      orig->bands != decoded->bands)
    return fail(XV_EINVAL, "spectral angle: cubes differ in shape");
  memset(a, 0, sizeof *a);
  a->orig = orig->data;
  a->dec = decoded->data;
  a->dtype_orig = orig->dtype;
  a->dtype_dec = decoded->dtype;
  a->bands = (int)orig->bands;
  a->npix = orig->T * orig->H * orig->W;
  const int64_t want = (a->npix + kSaThreads - 1) / kSaThreads;
  *nblocks = (int)std::max<int64_t>(1, std::min<int64_t>(want, kSaMaxBlocks));
  return XV_OK;
}

// Bytes of scratch the kernels use for a grid of nblocks: per-block sums and
// counts, then the two totals.
size_t sa_scratch_bytes(int nblocks) { return (size_t)nblocks * 16 + 16; }

// Launches the kernels with their scratch at `mem` and returns the mean.
int sa_run(const xv_cube* orig, const xv_cube* decoded, SaArgs& a, int nblocks, void* mem,
           hipStream_t s, double* mean_rad, uint64_t* n_pixels) {
  a.part_sum = (double*)mem;
  a.part_n = (unsigned long long*)(a.part_sum + nblocks);
  a.out = (double*)(a.part_n + nblocks);
  hipError_t he;
  {
    const double ib = (orig->dtype == XV_U16 ? 2.0 : 4.0) + (decoded->dtype == XV_U16 ? 2.0 : 4.0);
    ProfScope ps(XV_K_QUALITY, s, (double)a.npix * a.bands * ib);
    he = launch_spectral_angle(a, nblocks, s);
  }
  uint64_t host[2] = {0, 0};
  if (he == hipSuccess) he = hipMemcpyAsync(host, a.out, 16, hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he != hipSuccess) return fail(XV_EHIP, "spectral angle: %s", hipGetErrorString(he));
  double sum;
  memcpy(&sum, &host[0], 8);
  const uint64_t n = host[1];
  *mean_rad = n ? sum / (double)n : NAN;
  if (n_pixels) *n_pixels = n;
  return XV_OK;
}

// Device address of `scratch` on each device, looked up once per device
// with that device current (the host-side name of the array is not a device
// address).
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;

int scratch_address(void** out) {
  int dev = 0;
  XV_HIP(hipGetDevice(&dev), "current device");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((size_t)dev >= g_scratch_ptr.size()) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    XV_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "address of the scratch array");
    if (!ptr) return fail(XV_EHIP, "scratch array has no device address");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return XV_OK;
}

}  // namespace

extern "C" {

int xv_spectral_angle(const xv_cube* orig, const xv_cube* decoded, double* mean_rad,
                      uint64_t* n_pixels, void* hip_stream) {
  SaArgs a;
  int nblocks = 0;
  int rc = sa_setup(orig, decoded, mean_rad, &a, &nblocks);
  if (rc != XV_OK) return rc;
  hipStream_t s = (hipStream_t)hip_stream;
  void* mem = nullptr;
  hipError_t he = dev_alloc(&mem, sa_scratch_bytes(nblocks), s);
  if (he != hipSuccess) return fail(XV_ENOMEM, "spectral angle scratch: %s", hipGetErrorString(he));
  rc = sa_run(orig, decoded, a, nblocks, mem, s, mean_rad, n_pixels);
  dev_free(mem, s);
  return rc;
}

int xv_spectral_angle_noalloc(const xv_cube* orig, const xv_cube* decoded, double* mean_rad,
                              uint64_t* n_pixels, void* hip_stream) {
  SaArgs a;
  int nblocks = 0;
  int rc = sa_setup(orig, decoded, mean_rad, &a, &nblocks);
  if (rc != XV_OK) return rc;
  if (sa_scratch_bytes(nblocks) > kSaScratchBytes)
    return fail(XV_EINVAL, "spectral angle: %zu bytes of scratch needed, the static array "
                "holds %zu", sa_scratch_bytes(nblocks), kSaScratchBytes);
  void* mem = nullptr;
  if ((rc = scratch_address(&mem)) != XV_OK) return rc;
  return sa_run(orig, decoded, a, nblocks, mem, (hipStream_t)hip_stream, mean_rad, n_pixels);
}

}  // extern "C"
