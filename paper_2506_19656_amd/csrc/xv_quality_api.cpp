// xv_quality_api.cpp -- host side of the quality metrics reported beside
// PSNR: SSIM of the coded planes and the spectral angle of decoded cubes.
#include <math.h>
#include <string.h>

#include <algorithm>

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

int xv_spectral_angle(const xv_cube* orig, const xv_cube* decoded, double* mean_rad,
                      uint64_t* n_pixels, void* hip_stream) {
  if (!mean_rad) return fail(XV_EINVAL, "null output");
  int rc = check_cube(orig, "original");
  if (rc != XV_OK) return rc;
  if ((rc = check_cube(decoded, "decoded")) != XV_OK) return rc;
  if (orig->T != decoded->T || orig->H != decoded->H || orig->W != decoded->W ||
      orig->bands != decoded->bands)
    return fail(XV_EINVAL, "spectral angle: cubes differ in shape");
  hipStream_t s = (hipStream_t)hip_stream;
  SaArgs a;
  memset(&a, 0, sizeof a);
  a.orig = orig->data;
  a.dec = decoded->data;
  a.dtype_orig = orig->dtype;
  a.dtype_dec = decoded->dtype;
  a.bands = (int)orig->bands;
  a.npix = orig->T * orig->H * orig->W;
  const int64_t want = (a.npix + kSaThreads - 1) / kSaThreads;
  const int nblocks = (int)std::max<int64_t>(1, std::min<int64_t>(want, 4096));
  void* mem = nullptr;
  hipError_t he = dev_alloc(&mem, (size_t)nblocks * 16 + 16, s);
  if (he != hipSuccess) return fail(XV_ENOMEM, "spectral angle scratch: %s", hipGetErrorString(he));
  a.part_sum = (double*)mem;
  a.part_n = (unsigned long long*)(a.part_sum + nblocks);
  a.out = (double*)(a.part_n + nblocks);
  {
    const double ib = (orig->dtype == XV_U16 ? 2.0 : 4.0) + (decoded->dtype == XV_U16 ? 2.0 : 4.0);
    ProfScope ps(XV_K_QUALITY, s, (double)a.npix * a.bands * ib);
    he = launch_spectral_angle(a, nblocks, s);
  }
  uint64_t host[2] = {0, 0};
  if (he == hipSuccess) he = hipMemcpyAsync(host, a.out, 16, hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  dev_free(mem, s);
  if (he != hipSuccess) return fail(XV_EHIP, "spectral angle: %s", hipGetErrorString(he));
  double sum;
  memcpy(&sum, &host[0], 8);
  const uint64_t n = host[1];
  *mean_rad = n ? sum / (double)n : NAN;
  if (n_pixels) *n_pixels = n;
  return XV_OK;
}

}  // extern "C"
