/*
 * xv_oracle.h -- declarations of the CPU oracle (test infrastructure only;
 * see xv_oracle.c for what each function computes and which passage of the
 * paper, or which stated reading of it, it follows).
 */
#ifndef XV_ORACLE_H
#define XV_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define XVO_U16 0
#define XVO_F32 1
#define XVO_PAD_ZERO 0
#define XVO_PAD_REPEAT 1
#define XVO_FILL_NEAREST 0
#define XVO_FILL_FORWARD 1

typedef struct {
  int32_t bit_depth;    /* B, 8..12 */
  int32_t qp;           /* -6(B-8)..51 */
  int32_t block;        /* N in {4, 8, 16, 32} */
  int32_t search_range; /* R, 0..64 */
  int32_t gop;          /* closed GOP length, >= 1 */
  int32_t pad_mode;     /* XVO_PAD_* */
  int32_t fill_mode;    /* XVO_FILL_* */
  int32_t qpel;         /* 1: quarter-sample motion (R <= 31), 0: integer */
  int32_t intra;        /* 1: I blocks predicted by DC / planar from their
                           reconstructed neighbours, 0: constant 2^(B-1) */
  int32_t split;        /* 1: P blocks coded whole or as four N/2 blocks
                           (N >= 8, integer vectors, no intra modes) */
} xvo_params;

int xvo_selfcheck(void);
int xvo_check_params(const xvo_params* p);

void xvo_stats(const void* data, int dtype, int64_t T, int64_t H, int64_t W,
               int64_t Bn, double* mn, double* mx, int64_t* n_valid);
double xvo_filled_value(const void* data, int dtype, int64_t T, int64_t H,
                        int64_t W, int64_t Bn, int64_t t, int64_t y, int64_t x,
                        int64_t b, int fill_mode, double mn_b, int* is_valid);
int32_t xvo_normalize(double x, double mn, double mx, int B);
double xvo_denormalize(int32_t q, double mn, double mx, int B);
double xvo_cast_output(double v, int dtype);
int64_t xvo_source_band(int64_t g, int c, int64_t Bn, int pad_mode);
void xvo_make_frame(const void* data, int dtype, int64_t T, int64_t H,
                    int64_t W, int64_t Bn, const double* mn, const double* mx,
                    const xvo_params* p, int64_t g, int64_t t, int64_t Hp,
                    int64_t Wp, uint16_t* frame, uint8_t* valid);

void xvo_dct_matrix(int N, int32_t* M);
void xvo_forward_transform(int N, int B, const int32_t* r, int32_t* C);
int32_t xvo_iq_scale(int k);
int32_t xvo_q_scale(int k);
void xvo_quantize(int N, int B, int qp, int intra, const int32_t* C,
                  int16_t* lev);
void xvo_dequantize(int N, int B, int qp, const int16_t* lev, int32_t* d);
void xvo_inverse_transform(int N, int B, const int32_t* d, int32_t* r);

int xvo_ue_len(uint32_t k);
int xvo_se_len(int32_t v);
void xvo_scan_order(int N, int32_t* order);
uint32_t xvo_coef_bits(int N, const int16_t* lev);
uint32_t xvo_mv_bits(int mvx, int mvy, int pmx, int pmy);

void xvo_motion_search(const uint16_t* cur, const uint16_t* ref, int64_t Hp,
                       int64_t Wp, int N, int R, int nch, int64_t bx,
                       int64_t by, int32_t* best_dx, int32_t* best_dy,
                       uint32_t* best_sad);

int xvo_luma_filter(int frac, int tap);
int32_t xvo_interp_sample(const uint16_t* plane, int64_t Hp, int64_t Wp, int B,
                          int64_t xq, int64_t yq);
void xvo_subpel_refine(const uint16_t* cur, const uint16_t* ref, int64_t Hp,
                       int64_t Wp, int N, int B, int nch, int64_t bx, int64_t by,
                       int dx, int dy, int32_t* mvx, int32_t* mvy,
                       uint32_t* best_sad);

/* PCA of the bands (u16 cubes): exact integer sums, covariance, cyclic
 * Jacobi eigen-decomposition, projection and its inverse. */
int xvo_pca_moments(const uint16_t* data, int64_t npix, int64_t Bn, double* mean,
                    double* cov);
int xvo_pca_eigen(const double* cov, int64_t Bn, double* eigval, double* basis);
void xvo_pca_project(const uint16_t* data, int64_t npix, int64_t Bn, const double* mean,
                     const double* basis, int64_t j0, int64_t j1, float* out);
void xvo_pca_inverse(const float* pcs, int64_t npix, int64_t Bn, int64_t k,
                     const double* mean, const double* basis, int out_dtype, void* out);

/* Intra prediction of I pictures: reference samples of block (bx, by) of a
 * plane whose blocks before it in raster order are reconstructed, in the
 * substitution order (p[-1][2N-1] .. p[-1][0], p[-1][-1], p[0][-1] ..
 * p[2N-1][-1]), and the N x N prediction [y][x] of mode 0 (planar) or 1 (DC). */
void xvo_intra_refs(const uint16_t* rec_plane, int64_t Hp, int64_t Wp, int N, int B,
                    int64_t bx, int64_t by, int32_t* refs);
void xvo_intra_predict(const int32_t* refs, int N, int mode, int B, int32_t* pred);

/* Adaptive block size (split): the lambda of the whole/split choice in
 * 1/16 SAD units; splits is [frames][Hb][Wb] (1 = split), NULL without the
 * tool.  With the tool the vectors are [frames][2 Hb][2 Wb][2] (N/2 grid). */
int32_t xvo_split_lambda(int qp, int B);
/* 1 when the four N/2 blocks (SADs sads, vectors (ux, uy), z-order) cost
 * less than the whole block (SAD sad_whole, vector (vx, vy)). */
int xvo_split_choose(uint32_t sad_whole, int vx, int vy, const uint32_t* sads,
                     const int32_t* ux, const int32_t* uy, int32_t lam16);
int xvo_encode_gop(const void* data, int dtype, int64_t T, int64_t H,
                   int64_t W, int64_t Bn, const double* mn, const double* mx,
                   const xvo_params* p, int64_t g, int64_t t0, int64_t len,
                   uint16_t* frames, int16_t* levels, int8_t* mvs,
                   uint16_t* recon, uint32_t* coef_bits, uint32_t* mv_bits,
                   uint8_t* splits, uint64_t* sse, uint64_t* nvalid);
int xvo_decode_gop(const xvo_params* p, int64_t H, int64_t W, int64_t len,
                   const int16_t* levels, const int8_t* mvs, const uint8_t* splits,
                   uint16_t* recon);
int xvo_encode_cube(const void* data, int dtype, int64_t T, int64_t H,
                    int64_t W, int64_t Bn, const xvo_params* p, double* mn,
                    double* mx, uint16_t* frames, int16_t* levels, int8_t* mvs,
                    uint16_t* recon, uint32_t* coef_bits, uint32_t* mv_bits,
                    uint8_t* splits, uint64_t* sse, uint64_t* nvalid);
int xvo_decode_cube(const xvo_params* p, int64_t T, int64_t H, int64_t W,
                    int64_t Bn, const int16_t* levels, const int8_t* mvs,
                    const uint8_t* splits, uint16_t* recon);
void xvo_denormalize_cube(const uint16_t* recon, int64_t T, int64_t H,
                          int64_t W, int64_t Bn, int N, int B, const double* mn,
                          const double* mx, int out_dtype, void* out);

/* Bitstream: the rate proxy's Exp-Golomb codes written out (see the
 * comment above xvo_write_bitstream for the order).  nframes = G * T frames,
 * frame f = g * T + t, intra when t % gop == 0.  index receives the bit
 * offset of each of the 4 * Hb segments per frame. */
uint64_t xvo_bitstream_bits(int N, int64_t G, int64_t T, int gop, int64_t Hb,
                            int64_t Wb, int imodes, const uint8_t* splits,
                            const int16_t* levels, const int8_t* mvs);
int xvo_write_bitstream(int N, int64_t G, int64_t T, int gop, int64_t Hb,
                        int64_t Wb, int imodes, const uint8_t* splits,
                        const int16_t* levels, const int8_t* mvs, uint8_t* out,
                        uint64_t out_bytes, uint64_t* index);
int xvo_read_bitstream(int N, int64_t G, int64_t T, int gop, int64_t Hb,
                       int64_t Wb, int imodes, uint8_t* splits, const uint8_t* in,
                       uint64_t bits, int16_t* levels, int8_t* mvs, uint64_t* index);

double xvo_psnr(double peak, double sse, double n);
double xvo_psnr_int(int B, uint64_t sse, uint64_t n);
double xvo_bpppb(uint64_t bits, int64_t T, int64_t H, int64_t W, int64_t Bn);
void xvo_phys_sse(const void* data, int dtype, int64_t T, int64_t H, int64_t W,
                  int64_t Bn, const uint16_t* recon, int N, int B,
                  const double* mn, const double* mx, double* sse_out);

void xvo_ssim_window(double w[11]);
double xvo_ssim_plane(const uint16_t* a, const uint16_t* b, int64_t stride, int64_t H,
                      int64_t W, int B);
void xvo_ssim_bands(const uint16_t* frames, const uint16_t* recon, int64_t T, int64_t H,
                    int64_t W, int64_t Bn, int N, int B, double* out);
double xvo_spectral_angle(const void* orig, int dtype_o, const void* dec, int dtype_d,
                          int64_t T, int64_t H, int64_t W, int64_t Bn, uint64_t* n_out);

#ifdef __cplusplus
}
#endif
#endif
