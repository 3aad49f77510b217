// xv_pca.cpp -- host side of the principal components of the bands: the fit
// (moments on the GPU, then the Bn x Bn eigen-decomposition here), and the
// projection and inverse launches.
//
// Covariance and eigenvectors are a small fixed chain of IEEE binary64
// operations on exact integer sums, evaluated on the host so that every step
// is a correctly rounded operation (the GPU's binary64 square root is not):
//   m_b  = S_b / n,
//   C_bc = ((n Q_bc - S_b S_c) / n) / n    (numerator exact in 128 bits),
// then the cyclic Jacobi method (Golub and Van Loan, "Matrix Computations":
// the symmetric 2x2 Schur rotation, pairs (p, q) in row-cyclic order, sweeps
// until the squared off-diagonal sum is at most 1e-30 of the squared
// diagonal sum, or 60 sweeps), eigenvalues in decreasing order (first index
// on ties), each eigenvector's component of largest magnitude (first such)
// made positive.
#include <math.h>
#include <string.h>

#include <vector>

#include "xv_host.h"

using namespace xv;
using namespace xv::host;

struct xv_pca {
  int32_t bands;
  int64_t npix;
  double mean[XV_MAX_BANDS];
  double cov[XV_MAX_BANDS * XV_MAX_BANDS];
  double eigval[XV_MAX_BANDS];
  double basis[XV_MAX_BANDS * XV_MAX_BANDS];  // [b][j], column j = PC j
  void* dev;                                  // mean [bands] then basis [bands][bands]
  hipStream_t stream;
};

namespace {

// Row-major index of the upper-triangle sum (b <= c) in the moments layout.
int tri_index(int Bn, int b, int c) {
  if (b > c) std::swap(b, c);
  return b * Bn - b * (b - 1) / 2 + (c - b);
}

// The eigen-decomposition of the symmetric matrix a (n x n, row-major).
void jacobi_eigen(int n, const double* a, double* eigval, double* basis) {
  std::vector<double> A(a, a + (size_t)n * n), V((size_t)n * n, 0.0);
  for (int i = 0; i < n; i++) V[(size_t)i * n + i] = 1.0;
  auto at = [&](std::vector<double>& M, int r, int c) -> double& { return M[(size_t)r * n + c]; };
  for (int sweep = 0; sweep < 60; sweep++) {
    double off = 0.0, dia = 0.0;
    for (int p = 0; p < n; p++) {
      dia += at(A, p, p) * at(A, p, p);
      for (int q = p + 1; q < n; q++) off += at(A, p, q) * at(A, p, q);
    }
    if (off <= 1e-30 * dia) break;
    for (int p = 0; p < n - 1; p++)
      for (int q = p + 1; q < n; q++) {
        const double apq = at(A, p, q);
        if (apq == 0.0) continue;
        // t: the root of smaller magnitude of t^2 + 2 theta t - 1 = 0
        const double theta = (at(A, q, q) - at(A, p, p)) / (2.0 * apq);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(1.0 + theta * theta));
        const double c = 1.0 / sqrt(1.0 + t * t);
        const double s = t * c;
        for (int k = 0; k < n; k++) {  // columns p and q
          const double x = at(A, k, p), y = at(A, k, q);
          at(A, k, p) = c * x - s * y;
          at(A, k, q) = s * x + c * y;
        }
        for (int k = 0; k < n; k++) {  // rows p and q
          const double x = at(A, p, k), y = at(A, q, k);
          at(A, p, k) = c * x - s * y;
          at(A, q, k) = s * x + c * y;
        }
        for (int k = 0; k < n; k++) {  // accumulated rotations
          const double x = at(V, k, p), y = at(V, k, q);
          at(V, k, p) = c * x - s * y;
          at(V, k, q) = s * x + c * y;
        }
      }
  }
  std::vector<char> taken(n, 0);
  for (int j = 0; j < n; j++) {
    int best = -1;
    for (int i = 0; i < n; i++)
      if (!taken[i] && (best < 0 || at(A, i, i) > at(A, best, best))) best = i;
    taken[best] = 1;
    eigval[j] = at(A, best, best);
    int big = 0;
    for (int b = 1; b < n; b++)
      if (fabs(at(V, b, best)) > fabs(at(V, big, best))) big = b;
    const double sign = at(V, big, best) < 0.0 ? -1.0 : 1.0;
    for (int b = 0; b < n; b++) basis[(size_t)b * n + j] = sign * at(V, b, best);
  }
}

int check_same_pixels(const xv_cube* a, const xv_cube* b, const char* what) {
  if (a->T != b->T || a->H != b->H || a->W != b->W)
    return fail(XV_EINVAL, "%s: cubes differ in T, H or W", what);
  return XV_OK;
}

}  // namespace

extern "C" {

int xv_pca_fit(const xv_cube* in, void* hip_stream, xv_pca** out) {
  if (!out) return fail(XV_EINVAL, "null output handle");
  *out = nullptr;
  int rc = check_cube(in, "PCA input");
  if (rc != XV_OK) return rc;
  if (in->dtype != XV_U16) return fail(XV_EINVAL, "PCA is defined for u16 cubes");
  hipStream_t s = (hipStream_t)hip_stream;
  const int Bn = (int)in->bands;
  const int64_t npix = in->T * in->H * in->W;
  const int P = pca_sum_count(Bn);
  const int nb = pca_moment_blocks(npix);
  void* mem = nullptr;
  XV_HIP(dev_alloc(&mem, (size_t)nb * P * 8 + (size_t)P * 16, s), "PCA moment buffers");
  PcaMomArgs a{in->data, npix, Bn, (unsigned long long*)mem,
               (unsigned long long*)mem + (size_t)nb * P};
  std::vector<uint64_t> tot((size_t)P * 2);
  hipError_t he;
  {
    ProfScope ps(XV_K_PCA, s, (double)npix * Bn * 2.0);
    he = launch_pca_moments(a, nb, s);
  }
  if (he == hipSuccess)
    he = hipMemcpyAsync(tot.data(), a.total, (size_t)P * 16, hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  dev_free(mem, s);
  if (he != hipSuccess) return hip_fail(he, "PCA moments");

  xv_pca* p = new (std::nothrow) xv_pca();
  if (!p) return fail(XV_ENOMEM, "host allocation failed");
  memset(p, 0, sizeof *p);
  p->bands = Bn;
  p->npix = npix;
  p->stream = s;
  auto u128 = [&](int q) {
    return ((unsigned __int128)tot[2 * (size_t)q + 1] << 64) | tot[2 * (size_t)q];
  };
  const int tri = Bn * (Bn + 1) / 2;
  const double n = (double)npix;
  for (int b = 0; b < Bn; b++) p->mean[b] = (double)u128(tri + b) / n;
  for (int b = 0; b < Bn; b++)
    for (int c = 0; c < Bn; c++) {
      const unsigned __int128 Sb = u128(tri + b), Sc = u128(tri + c);
      const __int128 num = (__int128)((unsigned __int128)npix * u128(tri_index(Bn, b, c))) -
                           (__int128)(Sb * Sc);
      p->cov[b * Bn + c] = ((double)num / n) / n;
    }
  jacobi_eigen(Bn, p->cov, p->eigval, p->basis);
  he = dev_alloc(&p->dev, (size_t)(Bn + Bn * Bn) * sizeof(double), s);
  if (he != hipSuccess) {
    delete p;
    return hip_fail(he, "PCA basis buffer");
  }
  std::vector<double> host(Bn + Bn * Bn);
  memcpy(host.data(), p->mean, Bn * sizeof(double));
  memcpy(host.data() + Bn, p->basis, (size_t)Bn * Bn * sizeof(double));
  he = hipMemcpyAsync(p->dev, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he != hipSuccess) {
    dev_free(p->dev, s);
    delete p;
    return hip_fail(he, "PCA basis upload");
  }
  *out = p;
  return XV_OK;
}

int xv_pca_view(const xv_pca* p, int32_t* bands, double* mean, double* cov, double* eigval,
                double* basis) {
  if (!p) return fail(XV_EINVAL, "null PCA");
  const int Bn = p->bands;
  if (bands) *bands = Bn;
  if (mean) memcpy(mean, p->mean, Bn * sizeof(double));
  if (cov) memcpy(cov, p->cov, (size_t)Bn * Bn * sizeof(double));
  if (eigval) memcpy(eigval, p->eigval, Bn * sizeof(double));
  if (basis) memcpy(basis, p->basis, (size_t)Bn * Bn * sizeof(double));
  return XV_OK;
}

int xv_pca_project(const xv_pca* p, const xv_cube* in, int32_t j0, int32_t j1,
                   const xv_cube* pcs, void* hip_stream) {
  if (!p) return fail(XV_EINVAL, "null PCA");
  int rc = check_cube(in, "PCA input");
  if (rc != XV_OK) return rc;
  if ((rc = check_cube(pcs, "PCA output")) != XV_OK) return rc;
  if (in->dtype != XV_U16 || in->bands != p->bands)
    return fail(XV_EINVAL, "PCA input must be the u16 band layout the PCA was fitted on");
  if (j0 < 0 || j1 <= j0 || j1 > p->bands)
    return fail(XV_EINVAL, "PC range %d..%d outside 0..%d", j0, j1, p->bands);
  if (pcs->dtype != XV_F32 || pcs->bands != j1 - j0)
    return fail(XV_EINVAL, "PCA output must be f32 with j1 - j0 bands");
  if ((rc = check_same_pixels(in, pcs, "PCA projection")) != XV_OK) return rc;
  hipStream_t s = (hipStream_t)hip_stream;
  const int64_t npix = in->T * in->H * in->W;
  PcaProjArgs a{in->data, npix, p->bands, j0, j1, (const double*)p->dev,
                (const double*)p->dev + p->bands, pcs->data};
  ProfScope ps(XV_K_PCA, s, (double)npix * (p->bands * 2.0 + (j1 - j0) * 4.0));
  XV_HIP(launch_pca_project(a, s), "PCA projection kernel");
  return XV_OK;
}

int xv_pca_inverse(const xv_pca* p, const xv_cube* pcs, const xv_cube* out, void* hip_stream) {
  if (!p) return fail(XV_EINVAL, "null PCA");
  int rc = check_cube(pcs, "PCs");
  if (rc != XV_OK) return rc;
  if ((rc = check_cube(out, "PCA inverse output")) != XV_OK) return rc;
  if (pcs->dtype != XV_F32 || pcs->bands > p->bands)
    return fail(XV_EINVAL, "PCs must be f32 with at most as many bands as the PCA");
  if (out->bands != p->bands) return fail(XV_EINVAL, "output must have the PCA's band count");
  if ((rc = check_same_pixels(pcs, out, "PCA inverse")) != XV_OK) return rc;
  hipStream_t s = (hipStream_t)hip_stream;
  const int64_t npix = pcs->T * pcs->H * pcs->W;
  PcaInvArgs a{pcs->data, npix, p->bands, (int32_t)pcs->bands, (const double*)p->dev,
               (const double*)p->dev + p->bands, out->dtype, out->data};
  const double ob = out->dtype == XV_U16 ? 2.0 : 4.0;
  ProfScope ps(XV_K_PCA, s, (double)npix * (pcs->bands * 4.0 + p->bands * ob));
  XV_HIP(launch_pca_inverse(a, s), "PCA inverse kernel");
  return XV_OK;
}

void xv_pca_free(xv_pca* p) {
  if (!p) return;
  if (p->dev) dev_free(p->dev, p->stream);
  delete p;
}

}  // extern "C"
