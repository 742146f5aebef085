/*
 * jxl_oracle.h -- plain FP64 CPU oracle for JPEG XL VarDCT pixel reconstruction.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The product path
 * (the HIP library and its binding) never links, imports or calls it, and the
 * two share no code, headers or tables.
 *
 * Every function follows the JPEG XL Committee Draft (ISO/IEC 18181 CD,
 * 2019-08-05) and cites the clause it implements.  Arithmetic is double
 * precision throughout ("real numbers", clause 5.4), except the one
 * expression the edge-preserving filter turns into an unsigned 8-bit guide
 * sample (J.2.2), which is evaluated in binary32 on purpose (see
 * orc_epf_pass).
 *
 * Conventions shared by all entry points:
 *   - images are planar, row-major, channel c in {0: X, 1: Y, 2: B};
 *   - a frame of xsize x ysize pixels has Wb = ceil(xsize/8) by Hb = ceil(ysize/8)
 *     blocks; coefficient planes are [8*Hb][8*Wb], per-block maps [Hb][Wb];
 *   - coefficient (x, y) of the varblock whose top-left block is (bx0, by0)
 *     is stored at plane position (8*bx0 + x, 8*by0 + y); x is the horizontal
 *     frequency index;
 *   - the DctSelect map follows C.5.4: only the entry at a varblock's
 *     top-left block is read; entries of other covered blocks are ignored.
 * Return values: 0 on success, a negative ORC_E_* code when the input is
 * ill-formed in the sense of the draft (C.5.4, C.6.1) or out of range.
 */
#ifndef JXL_ORACLE_H
#define JXL_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ORC_OK = 0,
  ORC_E_SIZE = -1,      /* xsize or ysize not positive */
  ORC_E_STRATEGY = -2,  /* DctSelect value outside the C.5.4 table or not supported */
  ORC_E_ALIGN = -3,     /* varblock not naturally aligned, out of bounds, or overlapping (C.5.4) */
  ORC_E_QUANT = -4,     /* quant field value outside [0, 256) (C.5.5) */
  ORC_E_DEQUANT = -5,   /* dequantization matrix entry not positive and finite (C.6.1) */
  ORC_E_PARAM = -6      /* frame parameter outside its range */
};

/* Transform types, numbered as in the C.5.4 table. */
enum {
  ORC_DCT8 = 0, ORC_IDENTITY = 1, ORC_DCT2 = 2, ORC_DCT4 = 3, ORC_DCT16 = 4,
  ORC_DCT32 = 5, ORC_DCT16X8 = 6, ORC_DCT8X16 = 7, ORC_DCT32X8 = 8,
  ORC_DCT8X32 = 9, ORC_DCT32X16 = 10, ORC_DCT16X32 = 11, ORC_DCT4X8 = 12,
  ORC_DCT8X4 = 13, ORC_AFV = 14
};

/* Encoding of one dequantization matrix (C.6.1), already read from the
 * stream: the encoding mode and the parameters that mode reads, per channel
 * X, Y, B.  Parameters a mode does not read are ignored. */
enum {
  ORC_DQ_LIBRARY = 0, ORC_DQ_IDENTITY = 1, ORC_DQ_DCT2 = 2, ORC_DQ_DCT4 = 3,
  ORC_DQ_DCT4X8 = 4, ORC_DQ_AFV = 5, ORC_DQ_DCT = 6, ORC_DQ_COPY = 7
};
typedef struct {
  int32_t mode;                 /* ORC_DQ_* */
  int32_t copy_from;            /* Copy: index of an earlier matrix */
  int32_t num_bands;            /* DCT, DCT4, DCT4x8: 2..17 distance bands */
  int32_t num_ecc_bands;        /* DCT, DCT4, DCT4x8: 1..8 eccentricity bands */
  double  dist_bands[3][17];    /* db */
  double  ecc_bands[3][8];      /* eb */
  double  params[3][6];         /* Identity 3, DCT2 6, DCT4 2, DCT4x8 1
                                   (dct4x8multipliers), AFV 2 (dct4multipliers) */
  double  afv_weights[3][8];    /* AFV */
} orc_dequant_encoding;

/* Frame parameters decoded from the headers (C.2, C.4, C.10, A.4.5, L.2). */
typedef struct {
  int32_t xsize, ysize;
  int32_t global_scale;        /* global_scale_minus_1 + 1 (C.4.2) */
  double  dc_mul[3];           /* mX_DC, mY_DC, mB_DC (C.4.1) */
  int32_t extra_levels[3];     /* extra_levels_xyb (C.5.2) */
  double  kx_dc, kb_dc;        /* DC chroma-from-luma factors, already as kX, kB (Annex G) */
  int32_t gab;                 /* loop_filter.gab (C.10) */
  double  gab_w1[3], gab_w2[3];/* Gaborish weights per channel (C.10) */
  int32_t epf_iters;           /* number of edge-preserving filter passes; 0 = off */
  double  epf_weight_min;
  double  epf_scale[3];
  double  epf_sharp_lut[8];
  double  epf_range_max, epf_range_mul, epf_quant_mul;
  int32_t epf_sigma_max;
  int32_t epf_sigma_shift;     /* kSigmaShift of J.2.4 */
  double  opsin_inv[9];        /* inverse opsin absorbance matrix, row-major (L.2) */
  double  opsin_bias[3];
  int32_t target_nits_div50;   /* ImageMetadata (A.4.5) */
  int32_t dc_smoothing;        /* adaptive DC smoothing of F.2; 0 = skipped */
  int32_t qco;                 /* loop_filter.qco (C.10): J.3 after the EPF passes */
  double  qco_interval_mul;    /* loop_filter.qco_interval_mul (C.10) */
  int32_t ac_prediction;       /* Annex H (kSkipPredictLF clear); 0 = skipped */
  int32_t noise;               /* kNoise (K.5); 0 = skipped */
  double  noise_lut[16];       /* C.4.8 LUT, each u(10) / 1024 */
  double  dot_colour_quant[3]; /* kColourQuant of K.2.1 (not given by the draft) */
  /* C.6.1 encodings of the 15 dequantization matrices, indexed by transform
   * type (C.5.4 numbering); NULL: all have their C.6.1.1 default encoding. */
  const orc_dequant_encoding* dq_enc;
  /* C.5.2 DcQuantField, float [3][Hb][Wb]: the dequantization range of each
   * DC sample (F.2 smoothing, J.3 LLF clamp); NULL: dc_mul[c] /
   * 2^extra_levels[c] everywhere (the field of a DC plane whose decoded
   * deltas are all 0; with extra_levels 0, the field whatever the deltas). */
  const float* dc_quant_field;
} orc_params;

/* Fills the defaults the draft gives for every field (C.4, C.10, L.2, A.4.5). */
void orc_params_default(orc_params* p, int32_t xsize, int32_t ysize);

/* Varblock size in pixels of a transform type (I.2.5); returns 0 if unknown. */
int orc_varblock_size(int strategy, int32_t* bx, int32_t* by);

/* ---- transforms (Annex I) ---------------------------------------------- */
/* T_N (N in {1,2,4,8,16,32}): inverse 1-D transform of I.2.1 as a matrix,
 * out[n*N + k] = weight of input coefficient k in output sample n. */
int orc_idct_matrix(int32_t N, double* out);
/* F_N: forward 1-D transform of I.2.1 as a matrix, out[k*N + n]. */
int orc_fdct_matrix(int32_t N, double* out);
/* I(N, u), D(N, u), ScaleF(N, n, x) of I.2.6.1. */
double orc_scale_I(int32_t N, int32_t u);
double orc_scale_D(int32_t N, int32_t u);
double orc_scalef(int32_t N, int32_t n, int32_t x);
/* Inverse transform of one varblock (I.2.4): coefficients [by][bx] -> samples [by][bx]. */
/* The AFV basis of I.2.2 as a 16 x 16 row-major array (row i = basis vector i). */
void orc_afv_basis(double* out);
int orc_inverse_transform(int strategy, const double* coeffs, double* samples);
/* Forward transform of one varblock (I.2.3); used by round-trip pins only. */
int orc_forward_transform(int strategy, const double* samples, double* coeffs);
/* LLF coefficients from the downsampled (DC) image (I.2.7, N = 8):
 * dc [cy][cx] -> llf [cy][cx]. */
int orc_llf_from_dc(int strategy, const double* dc, double* llf);
/* Downsampled image from LF coefficients (I.2.6, N = 8): llf [cy][cx] -> dc [cy][cx]. */
int orc_dc_from_llf(int strategy, const double* llf, double* dc);

/* The same at N = 4 (Annex H): llf [cy][cx] -> cells [2cy][2cx] (8x8 types:
 * 2 x 2), and cells -> the top [2cy][2cx] coefficients (I.2.7, N = 4). */
int orc_dc2x2_from_llf(int strategy, const double* llf, double* cells);
int orc_llf2x2_from_dc2x2(int strategy, const double* cells, double* coeffs);
/* ---- dequantization (C.6.1, F.3) --------------------------------------- */
/* Default dequantization matrix of a transform type and channel, [by][bx]. */
int orc_dequant_matrix(int strategy, int c, double* out);
/* The matrix of a transform type and channel under the encodings enc[15]
 * (NULL: defaults), [by][bx]; ORC_E_DEQUANT when the encoding is not valid
 * for the type or an entry is not positive and finite. */
int orc_dequant_matrix_enc(int strategy, int c, const orc_dequant_encoding* enc, double* out);
/* The C.6.1.1 default encoding of a transform type (mode and parameters). */
int orc_default_encoding(int strategy, orc_dequant_encoding* out);

/* ---- reconstruction (F, G, I) ------------------------------------------ */
/* Quantized DC/AC planes and side maps -> XYB samples, cropped to xsize x ysize.
 * cfl_kx/cfl_kb: per 64x64 tile kX and kB of Annex G, [ceil(ysize/64)][ceil(xsize/64)]. */
/* Annex H image step: the smoothed 2x2-cell image [3][2Hb][2Wb] of a frame
 * from its DC samples [3][Hb][Wb] (after F.2 and the DC chroma from luma);
 * margin: each cell's |wa - s| - 1.7 dcq (the smoothing test's distance). */
void orc_ac_prediction_image(const orc_params* p, int32_t Wb, int32_t Hb,
                             const uint8_t* strategy, const double* dcq, double* out,
                             double* margin /* [3][2Hb][2Wb] or NULL */);
/* F.2 adaptive DC smoothing of a dequantized DC image [3][Hb][Wb], in place. */
void orc_dc_smooth(const orc_params* p, int32_t Wb, int32_t Hb, double* dcq);
int orc_reconstruct(const orc_params* p,
                    const int32_t* const ac[3], const int32_t* const dc[3],
                    const uint8_t* strategy, const uint8_t* qf_minus_1,
                    const float* cfl_kx, const float* cfl_kb,
                    double* xyb /* [3][ysize][xsize] */);

/* ---- loop filters (Annex J) -------------------------------------------- */
/* mul_table of J.2.4 for sigma in [0, 672]; entries below 16 are 0. */
int orc_epf_mul_table(int32_t sigma_shift, int32_t* table /* [673] */);
/* Weight(sad, mul) of J.2.4 as its binary32 value. */
float orc_epf_weight(int32_t sad, int32_t mul);
/* One edge-preserving filter pass (J.2) over a cropped XYB frame.
 * guide_out [3][ysize][xsize] and sigma_out [Hb][Wb] may be NULL. */
int orc_epf_pass(const orc_params* p, const uint8_t* strategy,
                 const uint8_t* qf_minus_1, const uint8_t* sharpness,
                 const double* in, double* out,
                 uint8_t* guide_out, int32_t* sigma_out);
/* Quantization constraint (J.3): orig is the input of the first filter
 * pass, filt the output of the last, out receives the constrained frame
 * (all [3][ysize][xsize]; out may not alias orig). */
int orc_qco(const orc_params* p, const uint8_t* strategy, const uint8_t* qf_minus_1,
            const double* orig, const double* filt, double* out);
/* K.3 patches, added in place: n placements of (x, y, xsize, ysize, offset
 * into samples), samples [3][ysize][xsize] integers per patch. */
int orc_patches(const orc_params* p, const int32_t* place, int32_t n, const int32_t* samples,
                double* xyb);
/* K.2 dots, added in place: n quantized dots of 10 integers (x, y, sigma_x,
 * sigma_y, angle, sign_intensity, intensity[3], is_circle). */
int orc_dots(const orc_params* p, const int32_t* dots, int32_t n, double* xyb);
/* K.4 splines, added in place: ContinuousIDCT of 32 coefficients at t; the
 * sampled centripetal Catmull-Rom sequence C of n control points (room for
 * 16 (n - 1) + 1; -1 if consecutive points coincide); the unit-arc-length
 * walk P over C (x, y, l, d per point; returns the count, *L the length);
 * and the rendering of n splines (offsets[n + 1] into pts (x, y) pairs,
 * dct[n][4][32] for X, Y, B, sigma; near: [H][W] flags or NULL). */
double orc_spline_idct(const float* dct, double t);
int32_t orc_spline_curve(const int32_t* pts, int32_t n, double* cx, double* cy);
int32_t orc_spline_walk(const double* cx, const double* cy, int32_t m, double* P, int32_t cap,
                        double* L);
int orc_splines(const orc_params* p, const int32_t* offsets, int32_t n, const int32_t* pts,
                const float* dct, double* xyb, uint8_t* near);
/* K.5.2 SplitMix64 and the three pseudorandom channels [3][gh][gw] of the
 * group with top-left pixel (x0, y0). */
uint64_t orc_splitmix64(uint64_t z);
/* One step of one of the eight XorShift128+ generators of K.5.2 on its state
 * (s0, s1), in place; returns batch[i] of that step. */
uint64_t orc_noise_step(uint64_t* s0, uint64_t* s1);
void orc_noise_channels(int32_t gw, int32_t gh, int32_t x0, int32_t y0, float* out);
/* K.5 noise over a cropped XYB frame (applied after Gaborish). */
int orc_noise(const orc_params* p, const double* in, double* out);
/* Gaborish (J.4). */
int orc_gaborish(const orc_params* p, const double* in, double* out);

/* ---- colour (Annex L) -------------------------------------------------- */
/* XYB -> linear RGB of L.2, divided by 255 ("[0,1]-scaled"). */
int orc_xyb_to_rgb(const orc_params* p, const double* xyb, double* rgb);
/* sRGB transfer function and rounding to 'bits' (8 or 16) per sample. */
int orc_quantize_srgb(int32_t bits, int64_t n, const double* lin, uint16_t* out);

/* ---- whole path -------------------------------------------------------- */
/* Reconstruct, epf_iters EPF passes, the quantization constraint (if p->qco
 * and at least one pass), Gaborish (if p->gab), noise (if p->noise),
 * XYB -> RGB.
 * rgb: [3][ysize][xsize] of [0,1]-scaled linear RGB. */
int orc_decode(const orc_params* p,
               const int32_t* const ac[3], const int32_t* const dc[3],
               const uint8_t* strategy, const uint8_t* qf_minus_1,
               const uint8_t* sharpness,
               const float* cfl_kx, const float* cfl_kb,
               double* rgb);

/* The same with patches (K.3) between the filters and Gaborish, and dots
 * (K.2) then splines (K.4) between Gaborish and the noise. */
int orc_decode_features(const orc_params* p,
                        const int32_t* const ac[3], const int32_t* const dc[3],
                        const uint8_t* strategy, const uint8_t* qf_minus_1,
                        const uint8_t* sharpness, const float* cfl_kx, const float* cfl_kb,
                        const int32_t* patch_place, int32_t n_patches,
                        const int32_t* patch_samples, const int32_t* dots, int32_t n_dots,
                        const int32_t* spline_offsets, int32_t n_splines,
                        const int32_t* spline_points, const float* spline_dct, double* rgb);
/* ---- JPEG1 direct rasterization (M.6) ---------------------------------- */
/* One component: dequantization (M.6.1, without the M.6.1.1 conditioning)
 * and IDCT_2D (M.6.2); qcoef int32 [8 hib][8 wib] in natural order per
 * block (index 8 u + v at row 8 by + u, column 8 bx + v), quant[64];
 * out [8 hib][8 wib]. */
int orc_jpeg1_component(const int32_t* qcoef, int32_t wib, int32_t hib, const int32_t* quant,
                        double* out);
/* M.6.3 block-gated Gaborish of one component's pixels [8 hib][8 wib], in
 * place; code: gab_weight1 * 1024, gab_weight2 * 1024, threshold * 16,
 * limit (the side channel's four bytes). */
int orc_jpeg1_gaborish(double* pix, int32_t wib, int32_t hib, const uint8_t* code);
/* M.6.4 linear 2x upsampling of n samples (mirrored ends), strided. */
void orc_upsample2(const double* in, int32_t n, size_t stride_in, double* out,
                   size_t stride_out);
/* M.6.4-M.6.6: upsampling, YCbCr -> RGB, crop; 1 (grey) or 3 components of
 * pixels [8 hib][8 wib] with sampling factors 1 or 2; rgb [3][ysize][xsize]. */
int orc_jpeg1_rasterize(int32_t ncomp, const double* const pix[3], const int32_t* wib,
                        const int32_t* hib, const int32_t* hs, const int32_t* vs, int32_t xsize,
                        int32_t ysize, double* rgb);
/* Number of OpenMP threads the oracle runs with (1 when built without OpenMP). */
int orc_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
