/*
 * jxl_oracle.c -- plain FP64 CPU oracle for JPEG XL VarDCT pixel reconstruction.
 *
 * TEST INFRASTRUCTURE ONLY: see jxl_oracle.h.  Written from the JPEG XL
 * Committee Draft (ISO/IEC 18181 CD, 2019-08-05).  Each function is the
 * draft's definition written out in the draft's order, with no blocking,
 * fusion or reordering; loops are plain and slow on purpose.  Where the draft
 * is silent, garbled or inconsistent, the reading taken is stated at the spot
 * and listed in the design notes of the repository.
 *
 * Parity status per function (pins live in tests/test_oracle_pins.py):
 *   transform matrices, inverse/forward transforms, LLF<->DC   pinned
 *   dequantization matrices                                     partially pinned
 *       (positivity, symmetry and closed-form band values only; the numerator
 *        reading of C.6.1 cannot be checked against anything but itself)
 *   reconstruct, gaborish, xyb_to_rgb, quantize_srgb            pinned
 *   edge-preserving filter                                      pinned by
 *       invariants and a step-edge closed form
 */
#include "jxl_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

/* ======================================================================= */
/* Defaults (C.4.1-C.4.3, C.10, L.2, A.4.5)                                */
/* ======================================================================= */

void orc_params_default(orc_params* p, int32_t xsize, int32_t ysize) {
  memset(p, 0, sizeof(*p));
  p->xsize = xsize;
  p->ysize = ysize;
  /* C.4.2 has no default; 1 is the smallest value the U32 can code. */
  p->global_scale = 1;
  /* C.4.1: weights {4096, 512, 256} times 1 / (global_scale * quant_dc),
   * here with global_scale = 1 and quant_dc = 1. */
  p->dc_mul[0] = 4096.0;
  p->dc_mul[1] = 512.0;
  p->dc_mul[2] = 256.0;
  /* C.4.3 + Annex G: x_factor_dc = b_factor_dc = 128. */
  p->kx_dc = (128.0 - 128.0) / 256.0;
  p->kb_dc = 0.935669 + (128.0 - 128.0) / 128.0;
  /* C.10 LoopFilter defaults. */
  p->gab = 1;
  for (int c = 0; c < 3; ++c) {
    p->gab_w1[c] = 0.115169525;
    p->gab_w2[c] = 0.061248592;
  }
  p->epf_iters = 1;
  p->epf_weight_min = 0.3;
  p->epf_scale[0] = 899.676941;
  p->epf_scale[1] = 111.965157;
  p->epf_scale[2] = 45.275791;
  for (int i = 0; i < 8; ++i) p->epf_sharp_lut[i] = i / 7.0;
  p->epf_range_max = 70.0;
  p->epf_range_mul = 12.6;
  p->epf_quant_mul = 20.0;
  p->epf_sigma_max = 170;
  p->epf_sigma_shift = 0;
  /* L.2 default inverse opsin absorbance matrix and biases. */
  static const double m[9] = {
      2542.56835937500000, -2326.53173828125000, 44.17734527587891,
      -698.04852294921875, 1012.71777343750000, -76.22974395751953,
      -827.36480712890625, 709.83502197265625,  451.38488769531250};
  memcpy(p->opsin_inv, m, sizeof(m));
  p->opsin_bias[0] = -0.00100549;
  p->opsin_bias[1] = -0.00100549;
  p->opsin_bias[2] = -0.00094081;
  p->target_nits_div50 = 5;  /* A.4.5 */
  p->qco = 0;                 /* C.10: qco defaults to false */
  p->qco_interval_mul = 0.5;
  p->ac_prediction = 0;
  p->noise = 0;  /* kNoise clear; the LUT is read only when it is set (C.4.8) */
  p->dot_colour_quant[0] = p->dot_colour_quant[1] = p->dot_colour_quant[2] = 0.0;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ======================================================================= */
/* Varblock geometry (C.5.4 table, I.2.5)                                  */
/* ======================================================================= */

/* I.2.5: "DCT N x M" has bxsize = max(8, N) and bysize = max(8, M); every other
 * transform covers 8 x 8.  The first number is read as the width. */
int orc_varblock_size(int s, int32_t* bx, int32_t* by) {
  static const int32_t w[15] = {8, 8, 8, 8, 16, 32, 16, 8, 32, 8, 32, 16, 8, 8, 8};
  static const int32_t h[15] = {8, 8, 8, 8, 16, 32, 8, 16, 8, 32, 16, 32, 8, 8, 8};
  if (s < 0 || s > 14) return 0;
  *bx = w[s];
  *by = h[s];
  return 1;
}

/* Transform types this oracle reconstructs: every C.5.4 value. */
static int supported(int s) { return s >= 0 && s <= 14; }

static int is_dct_family(int s) {
  return s == ORC_DCT8 || (s >= ORC_DCT16 && s <= ORC_DCT16X32);
}

/* ======================================================================= */
/* One-dimensional transforms (I.2.1 and the Annex R generator)            */
/* ======================================================================= */

/* The inverse transform of I.2.1 is the DCT-III with column k scaled:
 *   out[n] = sum_k s_N(k) * cos(pi * (2n + 1) * k / (2N)) * in[k],
 * s_N(0) = 1; s_8(k) = 1 / cos(k pi / 16) for the 8-point butterfly;
 * s_N(k) = 2 cos(k pi / (2N)) for the generated 2-, 4-, 16- and 32-point
 * transforms.  The forward transform is N times its inverse matrix:
 *   out[k] = r_N(k) * sum_n cos(pi * (2n + 1) * k / (2N)) * in[n],
 * r_N(0) = 1 and r_N(k) = 2 / s_N(k).  The tests pin both closed forms
 * against the butterfly and the generator's recursion. */
static double col_scale(int32_t N, int32_t k) {
  if (k == 0) return 1.0;
  if (N == 8) return 1.0 / cos(k * PI / 16.0);
  return 2.0 * cos(k * PI / (2.0 * N));
}

static int valid_n(int32_t N) {
  return N == 1 || N == 2 || N == 4 || N == 8 || N == 16 || N == 32;
}

int orc_idct_matrix(int32_t N, double* out) {
  if (!valid_n(N)) return ORC_E_PARAM;
  for (int32_t n = 0; n < N; ++n)
    for (int32_t k = 0; k < N; ++k)
      out[n * N + k] = col_scale(N, k) * cos(PI * (2 * n + 1) * k / (2.0 * N));
  return ORC_OK;
}

int orc_fdct_matrix(int32_t N, double* out) {
  if (!valid_n(N)) return ORC_E_PARAM;
  for (int32_t k = 0; k < N; ++k)
    for (int32_t n = 0; n < N; ++n) {
      double r = (k == 0) ? 1.0 : 2.0 / col_scale(N, k);
      out[k * N + n] = r * cos(PI * (2 * n + 1) * k / (2.0 * N));
    }
  return ORC_OK;
}

/* ======================================================================= */
/* Scale factors (I.2.6.1)                                                 */
/* ======================================================================= */

static double I8f(int32_t N, int32_t u) {
  double eps = (u == 0) ? sqrt(0.5) : 1.0;
  return sqrt(2.0 / N) * eps * cos(u * PI / (2.0 * N));
}
static double D8f(int32_t N, int32_t u) { return 1.0 / (N * I8f(N, u)); }

double orc_scale_I(int32_t N, int32_t u) { return N == 8 ? I8f(N, u) : D8f(N, u); }
double orc_scale_D(int32_t N, int32_t u) { return N == 8 ? D8f(N, u) : I8f(N, u); }

static double Cf(int32_t N, int32_t n, int32_t x) {
  if (n > N) return 1.0 / Cf(n, N, x);
  if (n == N) return 1.0;
  return cos(x * PI / (2.0 * N)) * Cf(N / 2, n, x);
}

double orc_scalef(int32_t N, int32_t n, int32_t x) {
  return sqrt((double)n * N) * orc_scale_D(N, x) * orc_scale_I(n, x) * Cf(N, n, x);
}

/* ======================================================================= */
/* Two-dimensional transforms (I.2.2, I.2.3, I.2.4)                        */
/* ======================================================================= */

/* Arrays are [rows][cols] = [y][x]; entry (x, y) of the draft is a[y * cols + x].
 *
 * Reading of I.2.2: coefficient (x, y) carries horizontal frequency x and
 * vertical frequency y for every size, so the 2-D inverse is
 * S = T_by * K * T_bx^T (rows transformed by T_by, columns by T_bx); the
 * draft's square form, which omits the final transpose, differs only by this
 * relabelling of a square coefficient array. */
static void idct_2d(int32_t bx, int32_t by, const double* K, double* S) {
  double Tx[32 * 32], Ty[32 * 32], tmp[32 * 32];
  orc_idct_matrix(bx, Tx);
  orc_idct_matrix(by, Ty);
  /* Column pass: tmp = T_by * K. */
  for (int32_t n = 0; n < by; ++n)
    for (int32_t x = 0; x < bx; ++x) {
      double acc = 0.0;
      for (int32_t k = 0; k < by; ++k) acc += Ty[n * by + k] * K[k * bx + x];
      tmp[n * bx + x] = acc;
    }
  /* Row pass: S = tmp * T_bx^T. */
  for (int32_t n = 0; n < by; ++n)
    for (int32_t m = 0; m < bx; ++m) {
      double acc = 0.0;
      for (int32_t k = 0; k < bx; ++k) acc += tmp[n * bx + k] * Tx[m * bx + k];
      S[n * bx + m] = acc;
    }
}

static void fdct_2d(int32_t bx, int32_t by, const double* S, double* K) {
  double Fx[32 * 32], Fy[32 * 32], tmp[32 * 32];
  orc_fdct_matrix(bx, Fx);
  orc_fdct_matrix(by, Fy);
  for (int32_t k = 0; k < by; ++k)
    for (int32_t x = 0; x < bx; ++x) {
      double acc = 0.0;
      for (int32_t n = 0; n < by; ++n) acc += Fy[k * by + n] * S[n * bx + x];
      tmp[k * bx + x] = acc;
    }
  for (int32_t k = 0; k < by; ++k)
    for (int32_t l = 0; l < bx; ++l) {
      double acc = 0.0;
      for (int32_t m = 0; m < bx; ++m) acc += tmp[k * bx + m] * Fx[l * bx + m];
      K[k * bx + l] = acc;
    }
}

/* AuxIDCT2x2(block, S) of I.2.4.2 on an 8 x 8 array: the top S x S cells are
 * replaced, the rest copied. */
static void aux_idct2x2(const double* blk, int S, double* res) {
  memcpy(res, blk, 64 * sizeof(double));
  int h = S / 2;
  for (int y = 0; y < h; ++y)
    for (int x = 0; x < h; ++x) {
      double c00 = blk[y * 8 + x];
      double c01 = blk[y * 8 + h + x];
      double c10 = blk[(h + y) * 8 + x];
      double c11 = blk[(h + y) * 8 + h + x];
      res[(2 * y) * 8 + 2 * x] = c00 + c01 + c10 + c11;
      res[(2 * y) * 8 + 2 * x + 1] = c00 + c01 - c10 - c11;
      res[(2 * y + 1) * 8 + 2 * x] = c00 - c01 + c10 - c11;
      res[(2 * y + 1) * 8 + 2 * x + 1] = c00 - c01 - c10 + c11;
    }
}

/* AuxDCT2x2(block, S) of I.2.3.2. */
static void aux_dct2x2(const double* blk, int S, double* res) {
  memcpy(res, blk, 64 * sizeof(double));
  int h = S / 2;
  for (int y = 0; y < h; ++y)
    for (int x = 0; x < h; ++x) {
      double c00 = blk[(2 * y) * 8 + 2 * x];
      double c01 = blk[(2 * y) * 8 + 2 * x + 1];
      double c10 = blk[(2 * y + 1) * 8 + 2 * x];
      double c11 = blk[(2 * y + 1) * 8 + 2 * x + 1];
      res[y * 8 + x] = (c00 + c01 + c10 + c11) / 4.0;
      res[y * 8 + h + x] = (c00 + c01 - c10 - c11) / 4.0;
      res[(h + y) * 8 + x] = (c00 - c01 + c10 - c11) / 4.0;
      res[(h + y) * 8 + h + x] = (c00 - c01 - c10 + c11) / 4.0;
    }
}

/* I.2.4.2: IDCT 2 x 2. */
static void inv_dct2(const double* K, double* S) {
  double a[64], b[64];
  aux_idct2x2(K, 2, a);
  aux_idct2x2(a, 4, b);
  aux_idct2x2(b, 8, S);
}

/* I.2.4.3: IDCT 4 x 4. */
static void inv_dct4(const double* K, double* S) {
  double dcs[64];
  aux_idct2x2(K, 2, dcs);
  for (int sy = 0; sy < 2; ++sy)
    for (int sx = 0; sx < 2; ++sx) {
      double blk[16], out[16];
      for (int iy = 0; iy < 4; ++iy)
        for (int ix = 0; ix < 4; ++ix)
          blk[iy * 4 + ix] = K[(sy + 2 * iy) * 8 + sx + 2 * ix];
      blk[0] = dcs[sy * 8 + sx];
      idct_2d(4, 4, blk, out);
      for (int l = 0; l < 4; ++l)
        for (int k = 0; k < 4; ++k) S[(4 * sy + l) * 8 + 4 * sx + k] = out[l * 4 + k];
    }
}

/* I.2.4.4: Identity. */
static void inv_identity(const double* K, double* S) {
  double dcs[64];
  aux_idct2x2(K, 2, dcs);
  for (int sy = 0; sy < 2; ++sy)
    for (int sx = 0; sx < 2; ++sx) {
      double block_dc = dcs[sy * 8 + sx];
      double residual_sum = 0.0;
      for (int iy = 0; iy < 4; ++iy)
        for (int ix = 0; ix < 4; ++ix) {
          if (ix == 0 && iy == 0) continue;
          residual_sum += K[(sy + 2 * iy) * 8 + sx + 2 * ix];
        }
      double s11 = block_dc - residual_sum / 16.0;
      S[(4 * sy + 1) * 8 + 4 * sx + 1] = s11;
      for (int iy = 0; iy < 4; ++iy)
        for (int ix = 0; ix < 4; ++ix) {
          if (ix == 1 && iy == 1) continue;
          S[(4 * sy + iy) * 8 + 4 * sx + ix] = K[(sy + 2 * iy) * 8 + sx + 2 * ix] + s11;
        }
      S[(4 * sy) * 8 + 4 * sx] = K[(sy + 2) * 8 + sx + 2] + s11;
    }
}

/* The 16 x 16 orthonormal AFV basis of I.2.2; a 4 x 4 block is a 16-vector
 * with entry (x, y) at index 4 y + x.  Reading: two rows print 17 entries;
 * row 4 loses a trailing zero and row 9 the zero at index 3, which makes the
 * basis orthonormal (to 1.4e-14, tested). */
static const double AFV_BASIS[16][16] = {
    {0.25, 0.25, 0.25, 0.25, 0.25, 0.25, 0.25, 0.25, 0.25, 0.25, 0.25, 0.25, 0.25, 0.25, 0.25,
     0.25},
    {0.876902929799142, 0.2206518106944235, -0.10140050393753763, -0.1014005039375375,
     0.2206518106944236, -0.10140050393753777, -0.10140050393753772, -0.10140050393753763,
     -0.10140050393753758, -0.10140050393753769, -0.1014005039375375, -0.10140050393753768,
     -0.10140050393753768, -0.10140050393753759, -0.10140050393753763, -0.10140050393753741},
    {0.0, 0.0, 0.40670075830260755, 0.44444816619734445, 0.0, 0.0, 0.19574399372042936,
     0.2929100136981264, -0.40670075830260716, -0.19574399372042872, 0.0, 0.11379074460448091,
     -0.44444816619734384, -0.29291001369812636, -0.1137907446044814, 0.0},
    {0.0, 0.0, -0.2125574805828748, 0.3085497062849767, 0.0, 0.4706702258572536,
     -0.1621205195722993, 0.0, -0.21255748058287047, -0.16212051957228327, -0.47067022585725277,
     -0.1464291867126764, 0.3085497062849487, 0.0, -0.1464291867126536, 0.4251149611657548},
    {0.0, -0.7071067811865474, 0.0, 0.0, 0.7071067811865476, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0,
     0.0, 0.0, 0.0, 0.0},
    {-0.4105377591765233, 0.6235485373547691, -0.06435071657946274, -0.06435071657946266,
     0.6235485373547694, -0.06435071657946284, -0.0643507165794628, -0.06435071657946274,
     -0.06435071657946272, -0.06435071657946279, -0.06435071657946266, -0.06435071657946277,
     -0.06435071657946277, -0.06435071657946273, -0.06435071657946274, -0.0643507165794626},
    {0.0, 0.0, -0.4517556589999482, 0.15854503551840063, 0.0, -0.04038515160822202,
     0.0074182263792423875, 0.39351034269210167, -0.45175565899994635, 0.007418226379244351,
     0.1107416575309343, 0.08298163094882051, 0.15854503551839705, 0.3935103426921022,
     0.0829816309488214, -0.45175565899994796},
    {0.0, 0.0, -0.304684750724869, 0.5112616136591823, 0.0, 0.0, -0.290480129728998,
     -0.06578701549142804, 0.304684750724884, 0.2904801297290076, 0.0, -0.23889773523344604,
     -0.5112616136592012, 0.06578701549142545, 0.23889773523345467, 0.0},
    {0.0, 0.0, 0.3017929516615495, 0.25792362796341184, 0.0, 0.16272340142866204,
     0.09520022653475037, 0.0, 0.3017929516615503, 0.09520022653475055, -0.16272340142866173,
     -0.35312385449816297, 0.25792362796341295, 0.0, -0.3531238544981624, -0.6035859033230976},
    {0.0, 0.0, 0.40824829046386274, 0.0, 0.0, 0.0, 0.0, -0.4082482904638628, -0.4082482904638635,
     0.0, 0.0, -0.40824829046386296, 0.0, 0.408248290463863, 0.408248290463863, 0.0},
    {0.0, 0.0, 0.1747866975480809, 0.0812611176717539, 0.0, 0.0, -0.3675398009862027,
     -0.307882213957909, -0.17478669754808135, 0.3675398009862011, 0.0, 0.4826689115059883,
     -0.08126111767175039, 0.30788221395790305, -0.48266891150598584, 0.0},
    {0.0, 0.0, -0.21105601049335784, 0.18567180916109802, 0.0, 0.0, 0.49215859013738733,
     -0.38525013709251915, 0.21105601049335806, -0.49215859013738905, 0.0, 0.17419412659916217,
     -0.18567180916109904, 0.3852501370925211, -0.1741941265991621, 0.0},
    {0.0, 0.0, -0.14266084808807264, -0.3416446842253372, 0.0, 0.7367497537172237,
     0.24627107722075148, -0.08574019035519306, -0.14266084808807344, 0.24627107722075137,
     0.14883399227113567, -0.04768680350229251, -0.3416446842253373, -0.08574019035519267,
     -0.047686803502292804, -0.14266084808807242},
    {0.0, 0.0, -0.13813540350758585, 0.3302282550303788, 0.0, 0.08755115000587084,
     -0.07946706605909573, -0.4613374887461511, -0.13813540350758294, -0.0794670660591026,
     0.49724647109535086, 0.12538059448563663, 0.3302282550303805, -0.4613374887461554,
     0.12538059448564315, -0.13813540350758452},
    {0.0, 0.0, -0.1743760259965106, 0.0702790691196284, 0.0, -0.2921026642334881,
     0.3623817333531167, 0.0, -0.1743760259965108, 0.36238173335311646, 0.29210266423348785,
     -0.4326608024727445, 0.07027906911962818, 0.0, -0.4326608024727457, 0.34875205199302267},
    {0.0, 0.0, 0.1135498731499337, -0.07417504595810355, 0.0, 0.19402893032594343,
     -0.435190496523228, 0.21918684838857466, 0.11354987314994257, -0.4351904965232251,
     0.5550443808910661, -0.25468277124066463, -0.07417504595810233, 0.2191868483885728,
     -0.25468277124066413, 0.1135498731499429},
};

void orc_afv_basis(double* out) {
  for (int i = 0; i < 16; ++i)
    for (int j = 0; j < 16; ++j) out[i * 16 + j] = AFV_BASIS[i][j];
}

/* AFV_IDCT of I.2.2: samples[i] = sum_j coefficients[j] * AFV_BASIS[j][i]. */
static void afv_idct(const double* c, double* out) {
  for (int i = 0; i < 16; ++i) {
    double acc = 0.0;
    for (int j = 0; j < 16; ++j) acc += c[j] * AFV_BASIS[j][i];
    out[i] = acc;
  }
}

/* AFV_DCT of I.2.2: coefficients[i] = sum_j samples[j] * AFV_BASIS[i][j]. */
static void afv_dct(const double* smp, double* out) {
  for (int i = 0; i < 16; ++i) {
    double acc = 0.0;
    for (int j = 0; j < 16; ++j) acc += smp[j] * AFV_BASIS[i][j];
    out[i] = acc;
  }
}

/* I.2.4.5: IDCT 8 x 4.  Two halves 4 wide and 8 tall; half x takes the
 * coefficients of columns x, x + 2, x + 4, x + 6 and fills pixel columns
 * 4 x .. 4 x + 3 (reading: the draft leaves this placement unstated); the two
 * DC values are coefficients (0, 0) +- (1, 0). */
static void inv_dct8x4(const double* K, double* S) {
  const double dcs[2] = {K[0] + K[1], K[0] - K[1]};
  for (int x = 0; x < 2; ++x) {
    double blk[32], out[32];
    for (int iy = 0; iy < 8; ++iy)
      for (int ix = 0; ix < 4; ++ix) blk[iy * 4 + ix] = K[iy * 8 + x + 2 * ix];
    blk[0] = dcs[x];
    idct_2d(4, 8, blk, out);
    for (int iy = 0; iy < 8; ++iy)
      for (int ix = 0; ix < 4; ++ix) S[iy * 8 + 4 * x + ix] = out[iy * 4 + ix];
  }
}

/* I.2.4.6: IDCT 4 x 8.  Two halves 8 wide and 4 tall; half y takes the
 * coefficients of rows y, y + 2, y + 4, y + 6 and fills pixel rows
 * 4 y .. 4 y + 3; the two DC values are coefficients (0, 0) +- (0, 1).
 * Reading: the printed dcs[x] inside the loop over y is dcs[y]. */
static void inv_dct4x8(const double* K, double* S) {
  const double dcs[2] = {K[0] + K[8], K[0] - K[8]};
  for (int y = 0; y < 2; ++y) {
    double blk[32], out[32];
    for (int iy = 0; iy < 4; ++iy)
      for (int ix = 0; ix < 8; ++ix) blk[iy * 8 + ix] = K[(y + 2 * iy) * 8 + ix];
    blk[0] = dcs[y];
    idct_2d(8, 4, blk, out);
    for (int iy = 0; iy < 4; ++iy)
      for (int ix = 0; ix < 8; ++ix) S[(4 * y + iy) * 8 + ix] = out[iy * 8 + ix];
  }
}

/* I.2.4.7: AFV.  The four quarter DCs come from 4 x coefficients (0, 0),
 * (1, 0), (0, 1), (1, 1) by a 2 x 2 Hadamard step; quarter (x, y) takes the
 * coefficients (x + 2 ix, y + 2 iy), its AFV_IDCT is mirrored horizontally
 * when x = 1 and vertically when y = 1. */
static void inv_afv(const double* K, double* S) {
  const double c1 = K[0] * 4.0, c2 = K[1] * 4.0, c3 = K[8] * 4.0, c4 = K[9] * 4.0;
  const double dcs[4] = {c1 + c2 + c3 + c4, c1 + c2 - c3 - c4, c1 - c2 + c3 - c4,
                         c1 - c2 - c3 + c4};
  for (int y = 0; y < 2; ++y)
    for (int x = 0; x < 2; ++x) {
      double c[16], out[16];
      for (int iy = 0; iy < 4; ++iy)
        for (int ix = 0; ix < 4; ++ix) c[iy * 4 + ix] = K[(y + 2 * iy) * 8 + x + 2 * ix];
      c[0] = dcs[y * 2 + x];
      afv_idct(c, out);
      for (int iy = 0; iy < 4; ++iy)
        for (int ix = 0; ix < 4; ++ix)
          S[(4 * y + iy) * 8 + 4 * x + ix] = out[(y ? 3 - iy : iy) * 4 + (x ? 3 - ix : ix)];
    }
}

int orc_inverse_transform(int s, const double* K, double* S) {
  int32_t bx, by;
  if (!supported(s) || !orc_varblock_size(s, &bx, &by)) return ORC_E_STRATEGY;
  if (s == ORC_DCT2) inv_dct2(K, S);
  else if (s == ORC_DCT4) inv_dct4(K, S);
  else if (s == ORC_IDENTITY) inv_identity(K, S);
  else if (s == ORC_DCT8X4) inv_dct8x4(K, S);
  else if (s == ORC_DCT4X8) inv_dct4x8(K, S);
  else if (s == ORC_AFV) inv_afv(K, S);
  else idct_2d(bx, by, K, S);
  return ORC_OK;
}

/* I.2.3.2: DCT 2 x 2. */
static void fwd_dct2(const double* S, double* K) {
  double a[64], b[64];
  aux_dct2x2(S, 8, a);
  aux_dct2x2(a, 4, b);
  aux_dct2x2(b, 2, K);
}

/* I.2.3.3: DCT 4 x 4. */
static void fwd_dct4(const double* S, double* K) {
  double tmp[64];
  for (int sy = 0; sy < 2; ++sy)
    for (int sx = 0; sx < 2; ++sx) {
      double blk[16], c[16];
      for (int l = 0; l < 4; ++l)
        for (int k = 0; k < 4; ++k) blk[l * 4 + k] = S[(4 * sy + l) * 8 + 4 * sx + k];
      fdct_2d(4, 4, blk, c);
      for (int iy = 0; iy < 4; ++iy)
        for (int ix = 0; ix < 4; ++ix) tmp[(sy + 2 * iy) * 8 + sx + 2 * ix] = c[iy * 4 + ix];
    }
  aux_dct2x2(tmp, 2, K);
}

/* I.2.3.4: Identity. */
static void fwd_identity(const double* S, double* K) {
  double tmp[64];
  for (int sy = 0; sy < 2; ++sy)
    for (int sx = 0; sx < 2; ++sx) {
      double block_dc = 0.0;
      for (int iy = 0; iy < 4; ++iy)
        for (int ix = 0; ix < 4; ++ix) block_dc += S[(4 * sy + iy) * 8 + 4 * sx + ix];
      block_dc /= 16.0;
      double s11 = S[(4 * sy + 1) * 8 + 4 * sx + 1];
      for (int iy = 0; iy < 4; ++iy)
        for (int ix = 0; ix < 4; ++ix) {
          if (ix == 1 && iy == 1) continue;
          tmp[(sy + 2 * iy) * 8 + sx + 2 * ix] = S[(4 * sy + iy) * 8 + 4 * sx + ix] - s11;
        }
      tmp[(sy + 2) * 8 + sx + 2] = tmp[sy * 8 + sx];
      tmp[sy * 8 + sx] = block_dc;
    }
  aux_dct2x2(tmp, 2, K);
}

/* I.2.3.5: DCT 8 x 4. */
static void fwd_dct8x4(const double* S, double* K) {
  for (int x = 0; x < 2; ++x) {
    double blk[32], c[32];
    for (int iy = 0; iy < 8; ++iy)
      for (int ix = 0; ix < 4; ++ix) blk[iy * 4 + ix] = S[iy * 8 + 4 * x + ix];
    fdct_2d(4, 8, blk, c);
    for (int iy = 0; iy < 8; ++iy)
      for (int ix = 0; ix < 4; ++ix) K[iy * 8 + x + 2 * ix] = c[iy * 4 + ix];
  }
  const double c0 = K[0], c1 = K[1];
  K[0] = (c0 + c1) * 0.5;
  K[1] = (c0 - c1) * 0.5;
}

/* I.2.3.6: DCT 4 x 8. */
static void fwd_dct4x8(const double* S, double* K) {
  for (int y = 0; y < 2; ++y) {
    double blk[32], c[32];
    for (int iy = 0; iy < 4; ++iy)
      for (int ix = 0; ix < 8; ++ix) blk[iy * 8 + ix] = S[(4 * y + iy) * 8 + ix];
    fdct_2d(8, 4, blk, c);
    for (int iy = 0; iy < 4; ++iy)
      for (int ix = 0; ix < 8; ++ix) K[(y + 2 * iy) * 8 + ix] = c[iy * 8 + ix];
  }
  const double c0 = K[0], c1 = K[8];
  K[0] = (c0 + c1) * 0.5;
  K[8] = (c0 - c1) * 0.5;
}

/* I.2.3.7: AFV. */
static void fwd_afv(const double* S, double* K) {
  for (int y = 0; y < 2; ++y)
    for (int x = 0; x < 2; ++x) {
      double smp[16], c[16];
      for (int iy = 0; iy < 4; ++iy)
        for (int ix = 0; ix < 4; ++ix)
          smp[(y ? 3 - iy : iy) * 4 + (x ? 3 - ix : ix)] = S[(4 * y + iy) * 8 + 4 * x + ix];
      afv_dct(smp, c);
      for (int iy = 0; iy < 4; ++iy)
        for (int ix = 0; ix < 4; ++ix) K[(y + 2 * iy) * 8 + x + 2 * ix] = c[iy * 4 + ix];
    }
  const double c1 = K[0] * 0.25, c2 = K[1] * 0.25, c3 = K[8] * 0.25, c4 = K[9] * 0.25;
  K[0] = (c1 + c2 + c3 + c4) * 0.25;
  K[1] = (c1 + c2 - c3 - c4) * 0.25;
  K[8] = (c1 - c2 + c3 - c4) * 0.25;
  K[9] = (c1 - c2 - c3 + c4) * 0.25;
}

int orc_forward_transform(int s, const double* S, double* K) {
  int32_t bx, by;
  if (!supported(s) || !orc_varblock_size(s, &bx, &by)) return ORC_E_STRATEGY;
  if (s == ORC_DCT2) fwd_dct2(S, K);
  else if (s == ORC_DCT4) fwd_dct4(S, K);
  else if (s == ORC_IDENTITY) fwd_identity(S, K);
  else if (s == ORC_DCT8X4) fwd_dct8x4(S, K);
  else if (s == ORC_DCT4X8) fwd_dct4x8(S, K);
  else if (s == ORC_AFV) fwd_afv(S, K);
  else fdct_2d(bx, by, S, K);
  return ORC_OK;
}

/* ======================================================================= */
/* LLF <-> downsampled image (I.2.6, I.2.7), N = 8                         */
/* ======================================================================= */

/* I.2.7.2 for the DCT family: C = DCT_2D(dc) (cy x cx), then
 * llf(x, y) = C(x, y) * ScaleF(cy, bysize, y) * ScaleF(cx, bxsize, x) / (cx * cy).
 * Reading: the division by cx * cy is not printed; without it I.2.7 would be
 * cx * cy times the inverse of I.2.6, which the draft says it is.
 * I.2.7.3 (N = 8) for the 8 x 8 transforms: llf = dc. */
int orc_llf_from_dc(int s, const double* dc, double* llf) {
  int32_t bx, by;
  if (!supported(s) || !orc_varblock_size(s, &bx, &by)) return ORC_E_STRATEGY;
  int32_t cx = bx / 8, cy = by / 8;
  if (!is_dct_family(s) || (cx == 1 && cy == 1)) {
    llf[0] = dc[0];
    return ORC_OK;
  }
  double C[16];
  fdct_2d(cx, cy, dc, C);
  for (int32_t y = 0; y < cy; ++y)
    for (int32_t x = 0; x < cx; ++x)
      llf[y * cx + x] = C[y * cx + x] * orc_scalef(cy, by, y) * orc_scalef(cx, bx, x) /
                        (double)(cx * cy);
  return ORC_OK;
}

/* I.2.6.2 (N = 8): scale the top cx x cy coefficients by
 * ScaleF(bysize, cy, y) * ScaleF(bxsize, cx, x) and take their cy x cx IDCT_2D.
 * I.2.6.3 for the 8 x 8 transforms: the single output is input(0, 0). */
int orc_dc_from_llf(int s, const double* llf, double* dc) {
  int32_t bx, by;
  if (!supported(s) || !orc_varblock_size(s, &bx, &by)) return ORC_E_STRATEGY;
  int32_t cx = bx / 8, cy = by / 8;
  if (!is_dct_family(s) || (cx == 1 && cy == 1)) {
    dc[0] = llf[0];
    return ORC_OK;
  }
  double L[16];
  for (int32_t y = 0; y < cy; ++y)
    for (int32_t x = 0; x < cx; ++x)
      L[y * cx + x] = llf[y * cx + x] * orc_scalef(by, cy, y) * orc_scalef(bx, cx, x);
  idct_2d(cx, cy, L, dc);
  return ORC_OK;
}

/* I.2.6 with N = 4: the 2cy x 2cx image of a varblock's 4x4-pixel cells from
 * its LLF coefficients (cy x cx), the other coefficients taken as 0.  DCT
 * family (I.2.6.2): the top 2cy x 2cx coefficients scaled by
 * ScaleF(bysize, 2cy, y) ScaleF(bxsize, 2cx, x), then the 2cy x 2cx IDCT_2D.
 * 8x8 types (I.2.6.3): the four cells take the DC. */
int orc_dc2x2_from_llf(int s, const double* llf, double* out) {
  int32_t bx, by;
  if (!supported(s) || !orc_varblock_size(s, &bx, &by)) return ORC_E_STRATEGY;
  if (!is_dct_family(s)) {
    for (int i = 0; i < 4; ++i) out[i] = llf[0];
    return ORC_OK;
  }
  const int32_t cx = bx / 8, cy = by / 8, cx4 = 2 * cx, cy4 = 2 * cy;
  double L[64];
  for (int32_t y = 0; y < cy4; ++y)
    for (int32_t x = 0; x < cx4; ++x)
      L[y * cx4 + x] = (x < cx && y < cy)
                           ? llf[y * cx + x] * orc_scalef(by, cy4, y) * orc_scalef(bx, cx4, x)
                           : 0.0;
  idct_2d(cx4, cy4, L, out);
  return ORC_OK;
}

/* I.2.7 with N = 4: the top 2cy x 2cx coefficients of a varblock from its
 * 2cy x 2cx image of 4x4-pixel cells.  DCT family (I.2.7.2 at N = 4, with the
 * division by the number of cells as in R2): C = DCT_2D(in), out(x, y) =
 * C(x, y) ScaleF(2cy, bysize, y) ScaleF(2cx, bxsize, x) / (4 cx cy).  8x8
 * types (I.2.7.3): AuxDCT2x2(in, 2) for Identity, DCT2, DCT4 and AFV; for
 * DCT8x4 and DCT4x8 the two printed forms.  Readings: the first form
 * printed for "DCT 8 x 4" (pairs along columns, the scaled differences down
 * the rows) is DCT8x4, whose DC pair is (0, 0) and (1, 0); the second, also
 * labelled "DCT 8 x 4", is DCT4x8 (DC pair (0, 0), (0, 1)), with its
 * "block11" read as coef4 = in(1, 1).  Only this assignment makes the
 * 4x4-cell means of the inverse transform equal the input (the property the
 * other types have), which the tests pin. */
int orc_llf2x2_from_dc2x2(int s, const double* in, double* out) {
  int32_t bx, by;
  if (!supported(s) || !orc_varblock_size(s, &bx, &by)) return ORC_E_STRATEGY;
  if (!is_dct_family(s)) {
    /* in / out are 2 x 2, entry (x, y) at [y * 2 + x] */
    const double c00 = in[0], c01 = in[1], c10 = in[2], c11 = in[3];
    if (s == ORC_DCT8X4 || s == ORC_DCT4X8) {
      const double sf = orc_scalef(2, 8, 1);
      if (s == ORC_DCT8X4) {
        const double dc0 = (c00 + c10) / 2, ac0 = (c00 - c10) / 2;
        const double dc1 = (c01 + c11) / 2, ac1 = (c01 - c11) / 2;
        out[0] = (dc0 + dc1) / 2;
        out[1] = (dc0 - dc1) / 2;
        out[2] = ac0 * sf;
        out[3] = ac1 * sf;
      } else {
        const double dc0 = (c00 + c01) / 2, ac0 = (c00 - c01) / 2;
        const double dc1 = (c10 + c11) / 2, ac1 = (c10 - c11) / 2;
        out[0] = (dc0 + dc1) / 2;
        out[2] = (dc0 - dc1) / 2;
        out[1] = ac0 * sf;
        out[3] = ac1 * sf;
      }
      return ORC_OK;
    }
    /* AuxDCT2x2(in, 2): block(x, y) = in[y * 2 + x] */
    out[0] = (c00 + c01 + c10 + c11) / 4;
    out[1] = (c00 + c01 - c10 - c11) / 4;
    out[2] = (c00 - c01 + c10 - c11) / 4;
    out[3] = (c00 - c01 - c10 + c11) / 4;
    return ORC_OK;
  }
  const int32_t cx4 = bx / 4, cy4 = by / 4;
  double C[64];
  fdct_2d(cx4, cy4, in, C);
  for (int32_t y = 0; y < cy4; ++y)
    for (int32_t x = 0; x < cx4; ++x)
      out[y * cx4 + x] = C[y * cx4 + x] * orc_scalef(cy4, by, y) * orc_scalef(cx4, bx, x) /
                         (double)(cx4 * cy4);
  return ORC_OK;
}

/* ======================================================================= */
/* Dequantization matrices (C.6.1, defaults C.6.1.1)                       */
/* ======================================================================= */

/* Default distance and eccentricity bands of the DCT-mode encodings (C.6.1.1),
 * per channel X, Y, B. */
static const double DB_DCT8[3][6] = {{5.0, 0.0, -0.4, -0.4, -0.4, -2.0},
                                     {1.1, 0.0, -0.3, -0.3, -0.3, -0.3},
                                     {1.0, -3.0, 0.0, 0.0, -1.0, -2.0}};
static const double DB_DCT4[3][4] = {{32.0, -0.4, 0.0, 0.0},
                                     {6.0, 0.0, 0.0, -0.0},
                                     {4.0, -5.0, -1.0, -1.0}};
static const double P_DCT4[3][2] = {{1.0, 1.0}, {0.7, 0.7}, {1.0, 1.0}};
static const double DB_DCT16[3][7] = {
    {3.1965020925735868, -1.8000777393353804, -0.39424529824571225, -0.33909377445710343,
     -0.6350101832695744, -0.90177264050827612, -1.5162099239887414},
    {0.77917081615440487, -0.57424582104194355, -0.90745813428471001, -0.64925837484843441,
     -0.35865440981033403, -0.21322389111877305, -0.27615025315725483},
    {0.22259376988644336, -3.0531423165804414, -0.2, -0.30687130033378396,
     -0.42708730624733904, -1.4856834539296244, -5.9209142884401604}};
static const double DB_DCT32[3][8] = {
    {0.47968775359573942, -1.025, -0.98, -0.9012, -0.4, -0.48819395464, -0.421064, -0.27},
    {0.22295421389982905, -0.8041958212306401, -0.7633036457487539, -0.55660379990111464,
     -0.49785304658857626, -0.43699592683512467, -0.40180866526242109, -0.27321683125358037},
    {0.11607457694128877, -3.060733579805728, -2.0413270132490346, -2.0235650159727417,
     -0.5495389509954993, -0.4, -0.4, -0.3}};
static const double DB_DCT16X8[3][7] = {{5.0, -0.7, -0.7, -0.2, -0.2, -0.2, -0.5},
                                        {1.0, -0.5, -0.5, -0.5, -0.2, -0.2, -0.2},
                                        {0.35, -1.4, -0.2, -0.5, -0.5, -1.5, -3.6}};
static const double DB_DCT32X8[3][8] = {
    {0.90897201669289496, -2.523575079652864, 1.5606102630460328, -0.6828050717528521,
     -14.770016895841904, -31.365240527393656, 0.565929254166433, 26.789646874558219},
    {0.3603042187746216, -0.11724474917749789, -0.85426302204085935, -0.5404181207241352,
     -0.45637619443533173, -0.82707923060149569, -1.09760551067614, -54.16057009483842},
    {0.25176400522276937, -10.060949304689093, -4.5316627381323995, -5.4569229849460807,
     -10.549754675878864, 1.7512906265092971, -1.6854706115725824, 3.3092762331901451}};
static const double EB_DCT32X8[3][4] = {
    {-0.40751133465833289, 2.2055690721475925, -1.4434547377534228, 2.0590289434445102},
    {0.12452072219659419, 0.065578935001406033, -0.14598888885596958, 0.12114139909222557},
    {0.0586589025020419, -2.2654958780302183, -4.6996221931893647, 1.8254498073137184}};
static const double DB_DCT32X16[3][8] = {
    {1.1280371559733287, -0.98868, -0.658, -0.42026, -0.22712, -0.2206, -0.226, -0.2},
    {0.38961075971152237, -0.62525308982767058, -0.83770786552491361, -0.79014862079498627,
     -0.2692727459704829, -0.38272769465388551, -0.2292422253091453, -0.20719098826199578},
    {0.098, -2.41, -0.23, -0.2, -0.4, -0.8, -0.4, -0.5}};
static const double P_IDENTITY[3][3] = {
    {221.50801256717435, 7087.151589594002, 4466.9924939259863},
    {29.535505378287006, 1454.6663024982124, 1368.041230099175},
    {9.2887405354132238, 23.982311358829531, 11.201853748207084}};
/* DCT4x8 mode (used by DCT4x8 and, transposed, by DCT8x4): four distance
 * bands per channel, two eccentricity bands of 0, per-channel multiplier 1.
 * Reading: the third channel's opening brace is lost in print. */
static const double DB_DCT4X8[3][4] = {
    {17.142628543359718, -0.16269623020744692, -0.31194253026666783, -0.2151140670773547},
    {4.6225628588812384, -0.82630200888366945, -1.0675229603596517, -0.17845290869168118},
    {0.81188546639482984, -0.6594385811273854, -0.050082094097871593, -2.6843722511996204}};
static const double P_DCT4X8[3] = {1.0, 1.0, 1.0};
/* AFV mode: eight afv_weights per channel and two dct4multipliers. */
static const double AFV_W[3][8] = {
    {6368.834817724610816928, 232.1096058872860158351, 415.663547479750900044,
     220.0720486370546864556, 329.818962738766012564, -0.9919974139384578, 0, -0.60},
    {1608.323575150649711025, 67.2724358236086, 89.06657498438612, 64.07248898359674,
     125.6541247697168638611, -2.2833978673775697, -0.14, -0.2485},
    {195.927828574730424638, 21.841306388764952, 18.5279466567289584105, 12.573868715940659,
     15.89916083965558, -0.41, -0.1608, 0}};
static const double AFV_P[3][2] = {{1.0, 1.0}, {1.0, 1.0}, {1.0, 1.0}};
static const double AFV_FREQS[16] = {
    0, 0, 0.8517778890324296, 5.37778436506804, 0, 0, 4.734747904497923, 5.449245381693219,
    1.6598270267479331, 4, 7.275749096817861, 10.423227632456525, 2.662932286148962,
    7.630657783650829, 8.962388608184032, 12.97166202570235};
static const double P_DCT2[3][6] = {{3840.0, 2560.0, 1280.0, 640.0, 480.0, 300.0},
                                    {960.0, 640.0, 320.0, 180.0, 140.0, 120.0},
                                    {640.0, 320.0, 128.0, 64.0, 32.0, 16.0}};

static double band_factor(double v) { return v > 0 ? (v + 1.0) : (1.0 / (1.0 - v)); }

/* interpolate() of C.6.1.  Reading: when the scaled position reaches the last
 * band (eccentricity 1 on the axes), the last band value is returned instead
 * of reading past the array. */
static double interpolate(double pos, double maxv, const double* bands, int len) {
  double scaled_pos = pos * (len - 1) / maxv;
  int idx = (int)floor(scaled_pos);
  if (idx >= len - 1) return bands[len - 1];
  double frac = scaled_pos - idx;
  double A = bands[idx], B = bands[idx + 1];
  return A * pow(B / A, frac);
}

/* Weights of the DCT encoding mode for an X-column by Y-row matrix.
 * Reading of the distance-band recurrence: bands[0] = db[0] and
 * bands[i] = bands[i - 1] * factor(db[i]) for 1 <= i < num_bands (the printed
 * loop writes index i + 1 and would leave index 1 unset). */
static void dct_weights(int X, int Y, const double* db, int nb, const double* eb, int ne,
                        double* w) {
  double dbands[17], ebands[9];
  dbands[0] = db[0];
  for (int i = 1; i < nb; ++i) dbands[i] = dbands[i - 1] * band_factor(db[i]);
  ebands[0] = 1.0;
  for (int i = 0; i < ne; ++i) ebands[i + 1] = ebands[i] * band_factor(eb ? eb[i] : 0.0);
  for (int y = 0; y < Y; ++y)
    for (int x = 0; x < X; ++x) {
      double fx = (double)x / X, fy = (double)y / Y;
      double dist = sqrt(fx * fx + fy * fy);
      double dm = interpolate(dist, sqrt(2.0), dbands, nb);
      /* eccentricity(0, 0) is 0 / 0; that entry is the DC slot and is never
       * used as a multiplier, so it is given multiplier 1. */
      double em = 1.0;
      if (x != 0 || y != 0) em = interpolate(fabs(fx - fy) / dist, 1.0, ebands, ne + 1);
      w[y * X + x] = dm * em;
    }
}

/* C.6.1.1: the default encoding of each transform type's matrix (the mode
 * the defaults are given in, and their parameters). */
int orc_default_encoding(int s, orc_dequant_encoding* e) {
  if (!supported(s)) return ORC_E_STRATEGY;
  memset(e, 0, sizeof(*e));
  const double* db = NULL;
  const double* eb = NULL;
  int nb = 0, ne = 0;
  for (int c = 0; c < 3; ++c) {
    switch (s) {
      case ORC_IDENTITY:
        e->mode = ORC_DQ_IDENTITY;
        for (int i = 0; i < 3; ++i) e->params[c][i] = P_IDENTITY[c][i];
        continue;
      case ORC_DCT2:
        e->mode = ORC_DQ_DCT2;
        for (int i = 0; i < 6; ++i) e->params[c][i] = P_DCT2[c][i];
        continue;
      case ORC_AFV:
        e->mode = ORC_DQ_AFV;
        for (int i = 0; i < 8; ++i) e->afv_weights[c][i] = AFV_W[c][i];
        e->params[c][0] = AFV_P[c][0];
        e->params[c][1] = AFV_P[c][1];
        continue;
      case ORC_DCT4:
        e->mode = ORC_DQ_DCT4;
        db = DB_DCT4[c]; nb = 4; ne = 2;
        e->params[c][0] = P_DCT4[c][0];
        e->params[c][1] = P_DCT4[c][1];
        break;
      case ORC_DCT4X8: case ORC_DCT8X4:
        e->mode = ORC_DQ_DCT4X8;
        db = DB_DCT4X8[c]; nb = 4; ne = 2;
        e->params[c][0] = P_DCT4X8[c];
        break;
      case ORC_DCT8: e->mode = ORC_DQ_DCT; db = DB_DCT8[c]; nb = 6; ne = 3; break;
      case ORC_DCT16: e->mode = ORC_DQ_DCT; db = DB_DCT16[c]; nb = 7; ne = 3; break;
      case ORC_DCT32: e->mode = ORC_DQ_DCT; db = DB_DCT32[c]; nb = 8; ne = 4; break;
      case ORC_DCT16X8: case ORC_DCT8X16:
        e->mode = ORC_DQ_DCT; db = DB_DCT16X8[c]; nb = 7; ne = 3; break;
      case ORC_DCT32X8: case ORC_DCT8X32:
        e->mode = ORC_DQ_DCT; db = DB_DCT32X8[c]; eb = EB_DCT32X8[c]; nb = 8; ne = 4; break;
      default:
        e->mode = ORC_DQ_DCT; db = DB_DCT32X16[c]; nb = 8; ne = 4; break;
    }
    e->num_bands = nb;
    e->num_ecc_bands = ne;
    for (int i = 0; i < nb; ++i) e->dist_bands[c][i] = db[i];
    for (int i = 0; i < ne; ++i) e->ecc_bands[c][i] = eb ? eb[i] : 0.0;
  }
  return ORC_OK;
}

/* The encoding matrix s is decoded with.  Readings: Library stands for the
 * default encoding of the matrix whose mode it is; Copy takes the encoding
 * (resolved the same way) of the earlier matrix it names, which is then
 * evaluated for the current transform type; matrices are indexed by
 * transform type in the C.5.4 order, Copy naming a smaller index. */
static int resolve_encoding(int s, const orc_dequant_encoding* enc, orc_dequant_encoding* out) {
  int idx = s;
  for (;;) {
    const orc_dequant_encoding* e = enc ? &enc[idx] : NULL;
    if (!e || e->mode == ORC_DQ_LIBRARY) return orc_default_encoding(idx, out);
    if (e->mode == ORC_DQ_COPY) {
      if (e->copy_from < 0 || e->copy_from >= idx) return ORC_E_DEQUANT;
      idx = e->copy_from;
      continue;
    }
    if (e->mode < 0 || e->mode > ORC_DQ_COPY) return ORC_E_DEQUANT;
    *out = *e;
    return ORC_OK;
  }
}

/* The weights matrix of transform type s (X columns by Y rows) for channel c
 * under the resolved encoding e (C.6.1). */
static int encoding_weights(int s, int c, const orc_dequant_encoding* e, double* w) {
  int32_t X, Y;
  orc_varblock_size(s, &X, &Y);
  const int banded = e->mode == ORC_DQ_DCT || e->mode == ORC_DQ_DCT4 || e->mode == ORC_DQ_DCT4X8;
  /* the Identity, DCT2, DCT4, DCT4x8 and AFV modes only define 64-entry matrices */
  if (e->mode != ORC_DQ_DCT && X * Y != 64) return ORC_E_DEQUANT;
  if (banded && (e->num_bands < 2 || e->num_bands > 17 || e->num_ecc_bands < 1 ||
                 e->num_ecc_bands > 8))
    return ORC_E_DEQUANT;
  const double* db = e->dist_bands[c];
  const double* eb = e->ecc_bands[c];
  const int nb = e->num_bands, ne = e->num_ecc_bands;
  const double* pc = e->params[c];
  if (e->mode == ORC_DQ_IDENTITY) {
    for (int i = 0; i < 64; ++i) w[i] = pc[0];
    w[0 * 8 + 1] = w[1 * 8 + 0] = pc[1];
    w[1 * 8 + 1] = pc[2];
  } else if (e->mode == ORC_DQ_DCT2) {
    /* Rectangles are half-open; "and symmetric" adds the mirror image across
     * the diagonal. */
    for (int y = 0; y < 8; ++y)
      for (int x = 0; x < 8; ++x) {
        int lo = x < y ? x : y, hi = x < y ? y : x;
        double v = 1.0;
        if (hi == 1 && lo == 0) v = pc[0];
        else if (hi == 1 && lo == 1) v = pc[1];
        else if (hi >= 2 && hi < 4 && lo < 2) v = pc[2];
        else if (hi >= 2 && hi < 4 && lo >= 2) v = pc[3];
        else if (hi >= 4 && lo < 4) v = pc[4];
        else if (hi >= 4 && lo >= 4) v = pc[5];
        w[y * 8 + x] = v;
      }
  } else if (e->mode == ORC_DQ_DCT4X8) {
    /* The 8-column by 4-row matrix of the band procedure, copied to (x, y)
     * from (x, y / 2); (0, 1) divided by the multiplier; transposed for
     * DCT8x4. */
    double w84[32], w48[64];
    dct_weights(8, 4, db, nb, eb, ne, w84);
    for (int y = 0; y < 8; ++y)
      for (int x = 0; x < 8; ++x) w48[y * 8 + x] = w84[(y / 2) * 8 + x];
    w48[1 * 8 + 0] /= pc[0];
    for (int y = 0; y < 8; ++y)
      for (int x = 0; x < 8; ++x) w[y * 8 + x] = s == ORC_DCT8X4 ? w48[x * 8 + y] : w48[y * 8 + x];
  } else if (e->mode == ORC_DQ_AFV) {
    /* Band values: bands[0] = afv_weights[4], bands[i] = bands[i - 1] *
     * factor(afv_weights[i + 4]) (reading: the printed factor reads index
     * i + 1 while its test reads i + 4; the band parameters are 5..7).  Each
     * value fills a 2 x 2 cell group (x, y) -> (2x .. 2x+1, 2y .. 2y+1). */
    const double* aw = e->afv_weights[c];
    double bands[4];
    bands[0] = aw[4];
    for (int i = 1; i < 4; ++i) bands[i] = bands[i - 1] * band_factor(aw[i + 4]);
    const double lo = 0.8517778890324296, hi = 12.1198851366699204;
    double w4[16];
    w4[0] = aw[0];
    w4[1 * 4 + 0] = aw[1]; /* set_weight(0, 1): x = 0, y = 1 */
    w4[0 * 4 + 1] = aw[2]; /* set_weight(1, 0) */
    w4[1 * 4 + 1] = aw[3];
    for (int y = 0; y < 4; ++y)
      for (int x = 0; x < 4; ++x) {
        if (x < 2 && y < 2) continue;
        w4[y * 4 + x] = interpolate(AFV_FREQS[y * 4 + x] - lo, hi, bands, 4);
      }
    for (int y = 0; y < 8; ++y)
      for (int x = 0; x < 8; ++x) w[y * 8 + x] = w4[(y / 2) * 4 + x / 2];
    w[0 * 8 + 1] *= pc[0];
    w[1 * 8 + 0] *= pc[0];
    w[1 * 8 + 1] *= pc[1];
  } else if (e->mode == ORC_DQ_DCT4) {
    double w4[16];
    dct_weights(4, 4, db, nb, eb, ne, w4);
    for (int y = 0; y < 8; ++y)
      for (int x = 0; x < 8; ++x) w[y * 8 + x] = w4[(y / 2) * 4 + x / 2];
    w[0 * 8 + 1] /= pc[0];
    w[1 * 8 + 0] /= pc[0];
    w[1 * 8 + 1] /= pc[1];
  } else {
    dct_weights(X, Y, db, nb, eb, ne, w);
  }
  return ORC_OK;
}

/* The numerators of transform type s (C.6.1), [Y][X]: 1 for AFV, DCT2 and
 * Identity; otherwise I(N_x, f_x) I(N_y, f_y) / (X Y), where on a dimension
 * of 4-point transforms (both of DCT4, the rows of DCT4x8, the columns of
 * DCT8x4) N = 4 and f = pos / 2, else N = the dimension and f = pos
 * (reading of the printed index expression, which does not distinguish X
 * from Y or the 4-point case). */
static void numerators(int s, double* num) {
  int32_t X, Y;
  orc_varblock_size(s, &X, &Y);
  for (int32_t y = 0; y < Y; ++y)
    for (int32_t x = 0; x < X; ++x) {
      double v;
      if (s == ORC_AFV || s == ORC_DCT2 || s == ORC_IDENTITY) v = 1.0;
      else if (s == ORC_DCT4) v = orc_scale_I(4, x / 2) * orc_scale_I(4, y / 2) / 64.0;
      else if (s == ORC_DCT4X8) v = orc_scale_I(8, x) * orc_scale_I(4, y / 2) / 64.0;
      else if (s == ORC_DCT8X4) v = orc_scale_I(4, x / 2) * orc_scale_I(8, y) / 64.0;
      else v = orc_scale_I(X, x) * orc_scale_I(Y, y) / (double)(X * Y);
      num[y * X + x] = v;
    }
}

int orc_dequant_matrix_enc(int s, int c, const orc_dequant_encoding* enc, double* out) {
  int32_t bx, by;
  if (!supported(s) || !orc_varblock_size(s, &bx, &by)) return ORC_E_STRATEGY;
  if (c < 0 || c > 2) return ORC_E_PARAM;
  orc_dequant_encoding e;
  int st = resolve_encoding(s, enc, &e);
  if (st) return st;
  double w[32 * 32], num[32 * 32];
  st = encoding_weights(s, c, &e, w);
  if (st) return st;
  numerators(s, num);
  for (int i = 0; i < bx * by; ++i) {
    double v = num[i] / w[i];
    /* entry (0, 0) is never a multiplier (the DC comes from the DC image) */
    if (i != 0 && !(v > 0.0 && isfinite(v))) return ORC_E_DEQUANT;
    out[i] = v;
  }
  return ORC_OK;
}

int orc_dequant_matrix(int s, int c, double* out) {
  return orc_dequant_matrix_enc(s, c, NULL, out);
}

/* ======================================================================= */
/* Reconstruction: F.2, F.3, Annex G, I.2.7, I.2.4                         */
/* ======================================================================= */

/* 6.5: mirrored index into [0, size). */
static int32_t mirror(int32_t coord, int32_t size) {
  while (coord < 0 || coord >= size) {
    if (coord < 0) coord = -coord - 1;
    else coord = 2 * size - 1 - coord;
  }
  return coord;
}

typedef struct {
  int32_t bx0, by0; /* top-left block */
  int s;
} varblock;

/* Walks the DctSelect map in raster order (C.5.4): at every block not yet
 * covered, the stored value names the varblock whose top-left it is; the
 * varblock must be naturally aligned and inside the frame.  A varblock that
 * would cover an already covered block is ill-formed as well. */
static int scan_varblocks(int32_t Wb, int32_t Hb, const uint8_t* strategy, varblock* list,
                          int32_t* count, int32_t* owner /* [Hb*Wb] or NULL */) {
  uint8_t* covered = (uint8_t*)calloc((size_t)Wb * Hb, 1);
  if (!covered) return ORC_E_SIZE;
  int32_t n = 0;
  for (int32_t by = 0; by < Hb; ++by)
    for (int32_t bx = 0; bx < Wb; ++bx) {
      if (covered[by * Wb + bx]) continue;
      int s = strategy[by * Wb + bx];
      int32_t w, h;
      if (!supported(s) || !orc_varblock_size(s, &w, &h)) { free(covered); return ORC_E_STRATEGY; }
      int32_t cx = w / 8, cy = h / 8;
      if (bx % cx || by % cy || bx + cx > Wb || by + cy > Hb) { free(covered); return ORC_E_ALIGN; }
      for (int32_t j = 0; j < cy; ++j)
        for (int32_t i = 0; i < cx; ++i) {
          if (covered[(by + j) * Wb + bx + i]) { free(covered); return ORC_E_ALIGN; }
          covered[(by + j) * Wb + bx + i] = 1;
          if (owner) owner[(by + j) * Wb + bx + i] = n;
        }
      list[n].bx0 = bx;
      list[n].by0 = by;
      list[n].s = s;
      ++n;
    }
  free(covered);
  *count = n;
  return ORC_OK;
}

/* F.3 bias adjustment of a quantized AC value. */
static const double kOneBias[3] = {0.05465007330715401, 0.07005449891748593,
                                   0.049935103337343655};
static double ac_bias(int32_t q, int c) {
  if (abs(q) <= 1) return q * (1.0 - kOneBias[c]);
  return q - 0.145 / q;
}

static int check_params(const orc_params* p) {
  if (p->xsize <= 0 || p->ysize <= 0) return ORC_E_SIZE;
  if (p->global_scale < 1 || p->global_scale > (1 << 16)) return ORC_E_PARAM;
  if (p->epf_sigma_max < 0 || p->epf_sigma_max > 672) return ORC_E_PARAM;
  if (p->epf_sigma_shift < 0 || p->epf_sigma_shift > 8) return ORC_E_PARAM;
  if (p->epf_iters < 0 || p->target_nits_div50 < 1) return ORC_E_PARAM;
  /* J.2.5 divides by the sum of weights; the centre weight is exactly 1, so a
   * threshold above 1 would leave nothing to divide by. */
  if (!(p->epf_weight_min <= 1.0)) return ORC_E_PARAM;
  for (int c = 0; c < 3; ++c)
    if (p->extra_levels[c] < 0 || p->extra_levels[c] > 3) return ORC_E_PARAM;
  /* every real-valued field must be finite (a NaN would pass the range tests
   * above and then reach integer conversions) */
  const double* fin[] = {p->dc_mul, &p->kx_dc, &p->kb_dc, p->gab_w1, p->gab_w2,
                         &p->epf_weight_min, p->epf_scale, p->epf_sharp_lut, &p->epf_range_max,
                         &p->epf_range_mul, &p->epf_quant_mul, p->opsin_inv, p->opsin_bias,
                         &p->qco_interval_mul, p->noise_lut, p->dot_colour_quant};
  const int nfin[] = {3, 1, 1, 3, 3, 1, 3, 8, 1, 1, 1, 9, 3, 1, 16, 3};
  for (size_t k = 0; k < sizeof(nfin) / sizeof(nfin[0]); ++k)
    for (int i = 0; i < nfin[k]; ++i)
      if (!isfinite(fin[k][i])) return ORC_E_PARAM;
  /* the DcQuantField is a positive dequantization range */
  if (p->dc_quant_field) {
    const size_t n = 3 * (size_t)((p->xsize + 7) / 8) * ((p->ysize + 7) / 8);
    for (size_t i = 0; i < n; ++i)
      if (!(p->dc_quant_field[i] > 0.0f && isfinite(p->dc_quant_field[i]))) return ORC_E_PARAM;
  }
  return ORC_OK;
}

/* The dequantization range (DcQuantField of C.5.2) of DC sample (x, y) of
 * channel c. */
static double dc_range(const orc_params* p, int c, int32_t x, int32_t y) {
  const int32_t Wb = (p->xsize + 7) / 8, Hb = (p->ysize + 7) / 8;
  if (p->dc_quant_field) return p->dc_quant_field[((size_t)c * Hb + y) * Wb + x];
  return p->dc_mul[c] / (double)(1 << p->extra_levels[c]);
}

/* F.2 adaptive DC smoothing of the dequantized DC image, per channel, in
 * place: every sample away from the first and last row and column becomes the
 * 3x3 weighted average of the unsmoothed samples (centre 0.05226273532324128,
 * edge neighbours 0.20345139757231578, diagonal ones 0.0334829185968739) when
 * that average lies within 0.5 dcq of the sample, else keeps its value;
 * dcq is the sample's DcQuantField (C.5.2).  Reading: the smoothing precedes
 * the DC chroma from luma. */
void orc_dc_smooth(const orc_params* p, int32_t Wb, int32_t Hb, double* dcq) {
  const double wc = 0.05226273532324128, we = 0.20345139757231578, wd = 0.0334829185968739;
  double* src = (double*)malloc(sizeof(double) * Wb * Hb);
  if (!src) return;
  for (int c = 0; c < 3; ++c) {
    double* d = dcq + (size_t)c * Wb * Hb;
    memcpy(src, d, sizeof(double) * Wb * Hb);
    for (int32_t y = 1; y + 1 < Hb; ++y)
      for (int32_t x = 1; x + 1 < Wb; ++x) {
        const double q = dc_range(p, c, x, y);
        const double* r0 = src + (size_t)(y - 1) * Wb + x;
        const double* r1 = src + (size_t)y * Wb + x;
        const double* r2 = src + (size_t)(y + 1) * Wb + x;
        const double s = r1[0];
        const double wa = wc * s + we * (r0[0] + r1[-1] + r1[1] + r2[0]) +
                          wd * (r0[-1] + r0[1] + r2[-1] + r2[1]);
        if (s - 0.5 * q <= wa && wa <= s + 0.5 * q) d[(size_t)y * Wb + x] = wa;
      }
  }
  free(src);
}

/* Annex H, the image step (margin, if not NULL, receives for each cell the
 * distance |wa - s| - 1.7 dcq of its smoothing test, negative when taken):
 * per channel and per group of 32 x 32 blocks
 * (groups of 256 x 256 samples, 6.2; the DC2x2 image of a group of gw x gh
 * blocks is (2 gw + 4) x (2 gh + 4)), the 2x2 cells of each varblock from its
 * LLF (I.2.6, N = 4), a border of two cells from the ring of DC samples
 * around the group (mirrored at the frame edge, 6.5), then the adaptive
 * smoothing of every cell inside the border: the 3x3 weighted average
 * (0.12 centre, 0.2 edge, 0.02 diagonal neighbours) of the unsmoothed cells
 * replaces the cell when within 1.7 dcq of it.  The smoothed cells are
 * stored in out [3][2 Hb][2 Wb] (cell (2 bx + i, 2 by + j) of block (bx, by)).
 * dcq is the channel's DC multiplier (C.4.1 with the C.4.2 fields; not the
 * per-sample DcQuantField that F.2 uses).  Readings: the DC samples are the
 * ones the LLF is computed from (after F.2 smoothing and the DC chroma from
 * luma); "xsize x ysize" of a group counts blocks. */
void orc_ac_prediction_image(const orc_params* p, int32_t Wb, int32_t Hb,
                             const uint8_t* strategy, const double* dcq, double* out,
                             double* margin) {
  const int32_t W2 = 2 * Wb;
  double* img = (double*)malloc(sizeof(double) * 68 * 68);
  double* sm = (double*)malloc(sizeof(double) * 68 * 68);
  if (!img || !sm) { free(img); free(sm); return; }
  for (int c = 0; c < 3; ++c) {
    const double* d = dcq + (size_t)c * Wb * Hb;
    const double q = p->dc_mul[c];
    for (int32_t gy0 = 0; gy0 < Hb; gy0 += 32)
      for (int32_t gx0 = 0; gx0 < Wb; gx0 += 32) {
        const int32_t gw = Wb - gx0 < 32 ? Wb - gx0 : 32, gh = Hb - gy0 < 32 ? Hb - gy0 : 32;
        const int32_t iw = 2 * gw + 4;
        /* border ring, then the varblocks inside */
        for (int32_t by = gy0 - 1; by <= gy0 + gh; ++by)
          for (int32_t bx = gx0 - 1; bx <= gx0 + gw; ++bx) {
            if (by >= gy0 && by < gy0 + gh && bx >= gx0 && bx < gx0 + gw) continue;
            const double v = d[(size_t)mirror(by, Hb) * Wb + mirror(bx, Wb)];
            for (int j = 0; j < 2; ++j)
              for (int i = 0; i < 2; ++i)
                img[(2 + 2 * (by - gy0) + j) * iw + 2 + 2 * (bx - gx0) + i] = v;
          }
        for (int32_t by = gy0; by < gy0 + gh; ++by)
          for (int32_t bx = gx0; bx < gx0 + gw; ++bx) {
            const int s = strategy[by * Wb + bx];
            int32_t vbx, vby;
            orc_varblock_size(s, &vbx, &vby);
            const int32_t cx = vbx / 8, cy = vby / 8;
            if (bx % cx || by % cy) continue; /* not a top-left block */
            double D[16], L[16], out4[64];
            const int32_t lx = is_dct_family(s) ? cx : 1, ly = is_dct_family(s) ? cy : 1;
            for (int32_t j = 0; j < cy; ++j)
              for (int32_t i = 0; i < cx; ++i) D[j * cx + i] = d[(size_t)(by + j) * Wb + bx + i];
            orc_llf_from_dc(s, D, L);
            orc_dc2x2_from_llf(s, L, out4);
            for (int32_t j = 0; j < 2 * ly; ++j)
              for (int32_t i = 0; i < 2 * lx; ++i)
                img[(2 + 2 * (by - gy0) + j) * iw + 2 + 2 * (bx - gx0) + i] = out4[j * 2 * lx + i];
          }
        for (int32_t y = 2; y < 2 * gh + 2; ++y)
          for (int32_t x = 2; x < 2 * gw + 2; ++x) {
            const double* r0 = img + (y - 1) * iw + x;
            const double* r1 = img + y * iw + x;
            const double* r2 = img + (y + 1) * iw + x;
            const double sv = r1[0];
            const double wa = 0.12 * sv + 0.2 * (r0[0] + r1[-1] + r1[1] + r2[0]) +
                              0.02 * (r0[-1] + r0[1] + r2[-1] + r2[1]);
            sm[y * iw + x] = (sv - 1.7 * q <= wa && wa <= sv + 1.7 * q) ? wa : sv;
            if (margin)
              margin[(size_t)c * W2 * 2 * Hb + (size_t)(2 * gy0 + y - 2) * W2 + 2 * gx0 + x - 2] =
                  fabs(wa - sv) - 1.7 * q;
          }
        for (int32_t y = 0; y < 2 * gh; ++y)
          for (int32_t x = 0; x < 2 * gw; ++x)
            out[(size_t)c * W2 * 2 * Hb + (size_t)(2 * gy0 + y) * W2 + 2 * gx0 + x] =
                sm[(y + 2) * iw + x + 2];
      }
  }
  free(img);
  free(sm);
}

int orc_reconstruct(const orc_params* p, const int32_t* const ac[3], const int32_t* const dc[3],
                    const uint8_t* strategy, const uint8_t* qf_minus_1, const float* cfl_kx,
                    const float* cfl_kb, double* xyb) {
  int st = check_params(p);
  if (st) return st;
  const int32_t W = p->xsize, H = p->ysize;
  const int32_t Wb = (W + 7) / 8, Hb = (H + 7) / 8;
  const int32_t PW = 8 * Wb;          /* padded plane width */
  const int32_t Wt = (W + 63) / 64;   /* CfL tiles per row */

  /* Dequantization matrices per transform type and channel. */
  double (*dq)[3][1024] = (double (*)[3][1024])malloc(sizeof(double) * 15 * 3 * 1024);
  if (!dq) return ORC_E_SIZE;
  for (int s = 0; s < 15; ++s)
    for (int c = 0; c < 3; ++c) {
      st = orc_dequant_matrix_enc(s, c, p->dq_enc, dq[s][c]);
      if (st) { free(dq); return st; }
    }

  /* F.2: dequantized DC, then Annex G on the DC with the DC factors. */
  double* dcq = (double*)malloc(sizeof(double) * 3 * Wb * Hb);
  varblock* list = (varblock*)malloc(sizeof(varblock) * Wb * Hb);
  double* pad = (double*)malloc(sizeof(double) * 3 * PW * 8 * Hb);
  if (!dcq || !list || !pad) { free(dq); free(dcq); free(list); free(pad); return ORC_E_SIZE; }
  for (int c = 0; c < 3; ++c)
    for (int32_t i = 0; i < Wb * Hb; ++i)
      dcq[c * Wb * Hb + i] = p->dc_mul[c] * dc[c][i] / (double)(1 << p->extra_levels[c]);
  if (p->dc_smoothing) orc_dc_smooth(p, Wb, Hb, dcq);
  for (int32_t i = 0; i < Wb * Hb; ++i) {
    double Y = dcq[1 * Wb * Hb + i];
    dcq[0 * Wb * Hb + i] += p->kx_dc * Y;
    dcq[2 * Wb * Hb + i] += p->kb_dc * Y;
  }
  /* Annex H: the smoothed 2x2-cell image, when AC prediction is on */
  double* pred = NULL;
  if (p->ac_prediction) {
    pred = (double*)malloc(sizeof(double) * 3 * 4 * (size_t)Wb * Hb);
    if (!pred) { free(dq); free(dcq); free(list); free(pad); return ORC_E_SIZE; }
  }

  int32_t nvb = 0;
  /* The quant field values are bytes, inside the [0, 256) range of C.5.5. */
  st = scan_varblocks(Wb, Hb, strategy, list, &nvb, NULL);
  if (st) { free(dq); free(dcq); free(list); free(pad); free(pred); return st; }
  if (pred) orc_ac_prediction_image(p, Wb, Hb, strategy, dcq, pred, NULL);

#pragma omp parallel for schedule(dynamic, 16)
  for (int32_t v = 0; v < nvb; ++v) {
    const varblock vb = list[v];
    int32_t bx, by;
    orc_varblock_size(vb.s, &bx, &by);
    const int32_t cx = bx / 8, cy = by / 8;
    /* C.5.5: AcMul of the varblock, from its top-left quant field value. */
    const double acmul =
        65536.0 / ((double)p->global_scale * (1.0 + qf_minus_1[vb.by0 * Wb + vb.bx0]));
    /* Annex G: the 64 x 64 region containing the varblock. */
    const int32_t tile = (vb.by0 * 8 / 64) * Wt + vb.bx0 * 8 / 64;
    const double kx = cfl_kx[tile], kb = cfl_kb[tile];
    double K[3][1024];
    for (int c = 0; c < 3; ++c) {
      /* F.3: bias, AcMul, dequantization matrix for every HF coefficient. */
      for (int32_t y = 0; y < by; ++y)
        for (int32_t x = 0; x < bx; ++x) {
          int32_t q = ac[c][(size_t)(8 * vb.by0 + y) * PW + 8 * vb.bx0 + x];
          K[c][y * bx + x] = ac_bias(q, c) * acmul * dq[vb.s][c][y * bx + x];
        }
      /* F.2 last paragraph + I.2.7: the LLF corner from the DC samples. */
      double D[16], L[16];
      for (int32_t j = 0; j < cy; ++j)
        for (int32_t i = 0; i < cx; ++i)
          D[j * cx + i] = dcq[c * Wb * Hb + (vb.by0 + j) * Wb + vb.bx0 + i];
      orc_llf_from_dc(vb.s, D, L);
      for (int32_t y = 0; y < cy; ++y)
        for (int32_t x = 0; x < cx; ++x) K[c][y * bx + x] = L[y * cx + x];
    }
    /* Annex G on the AC coefficients, with the tile's factors. */
    for (int32_t y = 0; y < by; ++y)
      for (int32_t x = 0; x < bx; ++x) {
        if (x < cx && y < cy) continue;
        double Y = K[1][y * bx + x];
        K[0][y * bx + x] += kx * Y;
        K[2][y * bx + x] += kb * Y;
      }
    /* Annex H: the top (2 lx) x (2 ly) coefficients from the varblock's cells
     * of the smoothed image (I.2.7, N = 4) are added, the LLF corner (lx x ly)
     * excepted.  Reading: the cells come from DC samples that already carry
     * the DC chroma from luma, so the sums are added after Annex G. */
    if (pred) {
      const int32_t lx = is_dct_family(vb.s) ? cx : 1, ly = is_dct_family(vb.s) ? cy : 1;
      for (int c = 0; c < 3; ++c) {
        double cell[64], P[64];
        for (int32_t j = 0; j < 2 * ly; ++j)
          for (int32_t i = 0; i < 2 * lx; ++i)
            cell[j * 2 * lx + i] =
                pred[(size_t)c * 4 * Wb * Hb + (size_t)(2 * vb.by0 + j) * 2 * Wb + 2 * vb.bx0 + i];
        orc_llf2x2_from_dc2x2(vb.s, cell, P);
        for (int32_t y = 0; y < 2 * ly; ++y)
          for (int32_t x = 0; x < 2 * lx; ++x)
            if (x >= lx || y >= ly) K[c][y * bx + x] += P[y * 2 * lx + x];
      }
    }
    /* Annex I: inverse transform, written at the varblock's pixels. */
    for (int c = 0; c < 3; ++c) {
      double S[1024];
      orc_inverse_transform(vb.s, K[c], S);
      for (int32_t y = 0; y < by; ++y)
        for (int32_t x = 0; x < bx; ++x)
          pad[(size_t)c * PW * 8 * Hb + (size_t)(8 * vb.by0 + y) * PW + 8 * vb.bx0 + x] =
              S[y * bx + x];
    }
  }
  /* 6.2: crop to xsize x ysize. */
  for (int c = 0; c < 3; ++c)
    for (int32_t y = 0; y < H; ++y)
      for (int32_t x = 0; x < W; ++x)
        xyb[(size_t)c * W * H + (size_t)y * W + x] =
            pad[(size_t)c * PW * 8 * Hb + (size_t)y * PW + x];
  free(dq);
  free(dcq);
  free(list);
  free(pad);
  free(pred);
  return ORC_OK;
}

/* ======================================================================= */
/* Mirroring (6.5)                                                         */
/* ======================================================================= */


/* ======================================================================= */
/* Edge-preserving filter (J.2)                                            */
/* ======================================================================= */

/* x >> s of 5.3.1: floor(x / 2^s). */
static int64_t shr_floor(int64_t x, int s) {
  int64_t d = (int64_t)1 << s;
  int64_t q = x / d;
  if ((x % d) != 0 && x < 0) --q;
  return q;
}

/* Weight(sad, mul) of J.2.4; MakeBinary32 of 5.2. */
float orc_epf_weight(int32_t sad, int32_t mul) {
  int64_t prescaled = (int64_t)(sad < 507 ? sad : 507) * 64;
  int64_t high16 = shr_floor(prescaled * mul, 16) + (127 << (23 - 16));
  uint32_t bits = (uint32_t)(high16 * 65536);
  float w;
  memcpy(&w, &bits, sizeof(w));
  return w;
}

/* mul_table of J.2.4.  kSigmaShift is not defined by the draft; it is a
 * parameter here (default 0).  Reading of the interpolation step: the printed
 * division is truncated toward zero (Idiv), so every entry is an integer. */
int orc_epf_mul_table(int32_t shift, int32_t* table) {
  const int gap = 4;
  int32_t mul = -32768;
  for (int i = 0; i <= 672; ++i) table[i] = 0;
  for (int32_t sigma = 16; sigma <= 672; sigma += gap) {
    for (; mul < 0; ++mul) {
      float w = orc_epf_weight(sigma >> shift, mul);
      if (w > 0.5f) break;
    }
    table[sigma] = mul;
  }
  for (int32_t sigma = 16; sigma < 672; sigma += gap) {
    int32_t diff = table[sigma + gap] - table[sigma];
    int32_t step = diff / gap; /* C division truncates toward zero: Idiv */
    for (int i = 1; i < gap; ++i) table[sigma + i] = table[sigma] + i * step;
  }
  return ORC_OK;
}

int orc_epf_pass(const orc_params* p, const uint8_t* strategy, const uint8_t* qf_minus_1,
                 const uint8_t* sharpness, const double* in, double* out,
                 uint8_t* guide_out, int32_t* sigma_out) {
  int st = check_params(p);
  if (st) return st;
  const int32_t W = p->xsize, H = p->ysize;
  const int32_t Wb = (W + 7) / 8, Hb = (H + 7) / 8;
  const size_t plane = (size_t)W * H;

  varblock* list = (varblock*)malloc(sizeof(varblock) * Wb * Hb);
  int32_t* owner = (int32_t*)malloc(sizeof(int32_t) * Wb * Hb);
  uint8_t* guide = (uint8_t*)malloc(3 * plane);
  double* brange = (double*)malloc(sizeof(double) * Wb * Hb);
  double* vrange = (double*)malloc(sizeof(double) * Wb * Hb);
  int32_t* sigma = (int32_t*)malloc(sizeof(int32_t) * Wb * Hb);
  int32_t mul_table[673];
  int32_t nvb = 0;
  if (!list || !owner || !guide || !brange || !vrange || !sigma) st = ORC_E_SIZE;
  if (!st) st = scan_varblocks(Wb, Hb, strategy, list, &nvb, owner);
  /* C.5.6: sharpness indexes the 8-entry epf_sharp_lut. */
  for (int32_t b = 0; !st && b < Wb * Hb; ++b)
    if (sharpness[b] > 7) st = ORC_E_PARAM;
  if (st) {
    free(list); free(owner); free(guide); free(brange); free(vrange); free(sigma);
    return st;
  }
  orc_epf_mul_table(p->epf_sigma_shift, mul_table);

  /* J.2.1: intensity_multiplier3 = cbrt(target_nits_div50 * 50 / 250). */
  const double im3 = cbrt(p->target_nits_div50 * 50.0 / 250.0);
  double minv[3];
  for (int c = 0; c < 3; ++c) minv[c] = (c != 0 ? 0.0 : -0.03) * im3;

  /* J.2.2: guide samples.  The draft stores them as unsigned 8-bit values and
   * does not say how the real value is rounded; reading: the clamped value is
   * floored, and this one expression is evaluated in binary32, the precision
   * of the GPU path, so that both take the integer decision alike. */
#pragma omp parallel for
  for (int32_t y = 0; y < H; ++y)
    for (int32_t x = 0; x < W; ++x)
      for (int c = 0; c < 3; ++c) {
        float sc = ((float)in[c * plane + (size_t)y * W + x] - (float)minv[c]) *
                   (float)p->epf_scale[c];
        float g = sc < 0.0f ? 0.0f : (sc > 255.0f ? 255.0f : sc);
        guide[c * plane + (size_t)y * W + x] = (uint8_t)floorf(g);
      }

  /* J.2.4: r[c] = max - min of `scaled` over each 8 x 8 block (the pixels of
   * the block inside the frame), all_r = max over channels. */
  for (int32_t by = 0; by < Hb; ++by)
    for (int32_t bx = 0; bx < Wb; ++bx) {
      double r = 0.0;
      for (int c = 0; c < 3; ++c) {
        double lo = INFINITY, hi = -INFINITY;
        for (int32_t y = 8 * by; y < 8 * by + 8 && y < H; ++y)
          for (int32_t x = 8 * bx; x < 8 * bx + 8 && x < W; ++x) {
            double sc = (in[c * plane + (size_t)y * W + x] - minv[c]) * p->epf_scale[c];
            if (sc < lo) lo = sc;
            if (sc > hi) hi = sc;
          }
        if (hi - lo > r) r = hi - lo;
      }
      brange[by * Wb + bx] = r;
    }
  /* range = the largest all_r within the varblock. */
  for (int32_t v = 0; v < nvb; ++v) {
    int32_t bx, by;
    orc_varblock_size(list[v].s, &bx, &by);
    double r = 0.0;
    for (int32_t j = 0; j < by / 8; ++j)
      for (int32_t i = 0; i < bx / 8; ++i) {
        double b = brange[(list[v].by0 + j) * Wb + list[v].bx0 + i];
        if (b > r) r = b;
      }
    for (int32_t j = 0; j < by / 8; ++j)
      for (int32_t i = 0; i < bx / 8; ++i) vrange[(list[v].by0 + j) * Wb + list[v].bx0 + i] = r;
  }
  /* sigma per block.  quant = 1 / AcMul is written as
   * global_scale * (1 + dv) / 65536, its exact value. */
  for (int32_t b = 0; b < Wb * Hb; ++b) {
    double range = vrange[b];
    if (range > p->epf_range_max) range = p->epf_range_max;
    double s = range * p->epf_range_mul * p->epf_sharp_lut[sharpness[b]];
    double quant = (double)p->global_scale * (1.0 + qf_minus_1[b]) / 65536.0;
    if (quant * p->epf_quant_mul < s) s = quant * p->epf_quant_mul;
    if ((double)p->epf_sigma_max < s) s = p->epf_sigma_max;
    sigma[b] = (int32_t)(s < 0 ? -floor(-s) : floor(s)); /* truncate */
  }

  /* J.2.3 + J.2.5.  Reading: mul_table is defined for sigma >= 16 only; a
   * pixel whose sigma is below 16 is passed through unfiltered. */
#pragma omp parallel for schedule(dynamic, 4)
  for (int32_t y = 0; y < H; ++y)
    for (int32_t x = 0; x < W; ++x) {
      const int32_t b = (y / 8) * Wb + x / 8;
      if (sigma[b] < 16) {
        for (int c = 0; c < 3; ++c)
          out[c * plane + (size_t)y * W + x] = in[c * plane + (size_t)y * W + x];
        continue;
      }
      const int32_t mul = mul_table[sigma[b]];
      int32_t sad[56];
      for (int i = 0; i < 56; ++i) sad[i] = 0;
      for (int c = 0; c < 3; ++c)
        for (int32_t cy = -3; cy <= 3; ++cy)
          for (int32_t cx = -3; cx <= 4; ++cx) {
            int32_t i = (cy + 3) * 8 + cx + 3;
            int32_t d = 0;
            for (int32_t iy = -1; iy <= 1; ++iy)
              for (int32_t ix = -1; ix <= 2; ++ix) {
                int32_t g0 = guide[c * plane + (size_t)mirror(y + iy, H) * W + mirror(x + ix, W)];
                int32_t g1 = guide[c * plane + (size_t)mirror(y + cy + iy, H) * W +
                                   mirror(x + cx + ix, W)];
                d += abs(g0 - g1);
              }
            sad[i] += d;
          }
      double weights[56];
      for (int i = 0; i < 56; ++i) {
        weights[i] = orc_epf_weight(sad[i], mul);
        if (weights[i] < p->epf_weight_min) weights[i] = 0.0;
      }
      double wsum[3] = {0, 0, 0}, sw[3] = {0, 0, 0};
      int i = 0;
      for (int32_t cy = -3; cy <= 3; ++cy)
        for (int32_t cx = -3; cx <= 4; ++cx) {
          double w = weights[i++];
          for (int c = 0; c < 3; ++c) {
            wsum[c] += in[c * plane + (size_t)mirror(y + cy, H) * W + mirror(x + cx, W)] * w;
            sw[c] += w;
          }
        }
      for (int c = 0; c < 3; ++c) out[c * plane + (size_t)y * W + x] = wsum[c] / sw[c];
    }

  if (guide_out) memcpy(guide_out, guide, 3 * plane);
  if (sigma_out) memcpy(sigma_out, sigma, sizeof(int32_t) * Wb * Hb);
  free(list); free(owner); free(guide); free(brange); free(vrange); free(sigma);
  return ORC_OK;
}

/* ======================================================================= */
/* Quantization constraint (J.3)                                           */
/* ======================================================================= */

/* The forward transforms of I.2.3 are unnormalized: followed by the inverse
 * transform of I.2.4 they give the samples times this gain (the number of
 * samples for the DCT family, 16 for DCT4 with its 4 x 4 sub-blocks, 32 for
 * the 4 x 8 halves of DCT4x8 and DCT8x4, 1 for the other types). */
static double forward_gain(int s, int32_t bx, int32_t by) {
  if (is_dct_family(s)) return (double)(bx * by);
  if (s == ORC_DCT4) return 16.0;
  if (s == ORC_DCT4X8 || s == ORC_DCT8X4) return 32.0;
  return 1.0;
}

/* For every varblock and channel: the residual filt - orig over the
 * varblock's samples goes through the varblock's forward transform (I.2.3,
 * divided by its gain, so that the coefficients are in the units of the
 * dequantized coefficients that I.2.4 maps back to samples);
 * its LLF corner is turned into DC samples (I.2.6); every DC sample and every
 * other coefficient is clamped to qco_interval_mul times its quantization
 * step on either side of 0; the DC samples go back to the LLF corner (I.2.7)
 * and the inverse transform (I.2.4) gives the residual that is added to
 * orig.  Readings:
 *   - the step of a coefficient outside the LLF corner is its dequantization
 *     matrix entry times AcMul (the factor F.3 multiplies a quantized value
 *     by), of a DC sample its DcQuantField (C.5.2);
 *   - samples of a varblock outside the frame were never filtered: their
 *     residual is 0, and only samples inside the frame are written;
 *   - the clamp acts on each channel's own coefficients (chroma from luma
 *     plays no part). */
int orc_qco(const orc_params* p, const uint8_t* strategy, const uint8_t* qf_minus_1,
            const double* orig, const double* filt, double* out) {
  int st = check_params(p);
  if (st) return st;
  if (!(p->qco_interval_mul >= 0.0)) return ORC_E_PARAM;
  const int32_t W = p->xsize, H = p->ysize;
  const int32_t Wb = (W + 7) / 8, Hb = (H + 7) / 8;
  double (*dq)[3][1024] = (double (*)[3][1024])malloc(sizeof(double) * 15 * 3 * 1024);
  varblock* list = (varblock*)malloc(sizeof(varblock) * Wb * Hb);
  if (!dq || !list) { free(dq); free(list); return ORC_E_SIZE; }
  for (int s = 0; s < 15 && !st; ++s)
    for (int c = 0; c < 3 && !st; ++c) st = orc_dequant_matrix_enc(s, c, p->dq_enc, dq[s][c]);
  int32_t nvb = 0;
  if (!st) st = scan_varblocks(Wb, Hb, strategy, list, &nvb, NULL);
  if (st) { free(dq); free(list); return st; }
  memcpy(out, filt, sizeof(double) * 3 * (size_t)W * H);
  const double m = p->qco_interval_mul;

#pragma omp parallel for schedule(dynamic, 16)
  for (int32_t v = 0; v < nvb; ++v) {
    const varblock vb = list[v];
    int32_t bx, by;
    orc_varblock_size(vb.s, &bx, &by);
    /* the LLF corner: cx x cy for the DCT family, the single (0, 0) otherwise */
    int32_t cx = bx / 8, cy = by / 8;
    if (!is_dct_family(vb.s)) cx = cy = 1;
    const double acmul =
        65536.0 / ((double)p->global_scale * (1.0 + qf_minus_1[vb.by0 * Wb + vb.bx0]));
    for (int c = 0; c < 3; ++c) {
      const size_t pl = (size_t)c * W * H;
      double R[1024], K[1024], S[1024], L[16], D[16];
      for (int32_t y = 0; y < by; ++y)
        for (int32_t x = 0; x < bx; ++x) {
          const int32_t gx = 8 * vb.bx0 + x, gy = 8 * vb.by0 + y;
          R[y * bx + x] =
              (gx < W && gy < H) ? filt[pl + (size_t)gy * W + gx] - orig[pl + (size_t)gy * W + gx]
                                 : 0.0;
        }
      orc_forward_transform(vb.s, R, K);
      const double g = forward_gain(vb.s, bx, by);
      for (int32_t y = 0; y < by; ++y)
        for (int32_t x = 0; x < bx; ++x) {
          const int32_t k = y * bx + x;
          K[k] /= g;
          if (x < cx && y < cy) {
            L[y * cx + x] = K[k];
          } else {
            const double t = m * dq[vb.s][c][k] * acmul;
            K[k] = fmin(fmax(K[k], -t), t);
          }
        }
      orc_dc_from_llf(vb.s, L, D);
      for (int32_t i = 0; i < cx * cy; ++i) {
        const double tq = m * dc_range(p, c, vb.bx0 + i % cx, vb.by0 + i / cx);
        D[i] = fmin(fmax(D[i], -tq), tq);
      }
      orc_llf_from_dc(vb.s, D, L);
      for (int32_t y = 0; y < cy; ++y)
        for (int32_t x = 0; x < cx; ++x) K[y * bx + x] = L[y * cx + x];
      orc_inverse_transform(vb.s, K, S);
      for (int32_t y = 0; y < by; ++y)
        for (int32_t x = 0; x < bx; ++x) {
          const int32_t gx = 8 * vb.bx0 + x, gy = 8 * vb.by0 + y;
          if (gx < W && gy < H)
            out[pl + (size_t)gy * W + gx] = orig[pl + (size_t)gy * W + gx] + S[y * bx + x];
        }
    }
  }
  free(dq);
  free(list);
  return ORC_OK;
}

/* ======================================================================= */
/* Patches (K.3)                                                           */
/* ======================================================================= */

/* K.3: every placement adds kChannelDequant[c] times its patch's samples at
 * its position.  place: n placements of 5 integers (x, y, xsize, ysize,
 * offset of the patch's samples in `samples`, which hold [3][ysize][xsize]
 * integers per patch); xsize, ysize at most 16 and the region inside the
 * frame (C.4.6), else ORC_E_PARAM. */
int orc_patches(const orc_params* p, const int32_t* place, int32_t n, const int32_t* samples,
                double* xyb) {
  static const double kChannelDequant[3] = {0.01615, 0.08875, 0.1922};
  const int32_t W = p->xsize, H = p->ysize;
  for (int32_t k = 0; k < n; ++k) {
    const int32_t* q = place + 5 * k;
    const int32_t x0 = q[0], y0 = q[1], xs = q[2], ys = q[3];
    if (xs < 1 || ys < 1 || xs > 16 || ys > 16 || x0 < 0 || y0 < 0 || x0 + xs > W || y0 + ys > H ||
        q[4] < 0)
      return ORC_E_PARAM;
  }
  for (int32_t k = 0; k < n; ++k) {
    const int32_t* q = place + 5 * k;
    const int32_t x0 = q[0], y0 = q[1], xs = q[2], ys = q[3];
    const int32_t* smp = samples + q[4];
    for (int c = 0; c < 3; ++c)
      for (int32_t iy = 0; iy < ys; ++iy)
        for (int32_t ix = 0; ix < xs; ++ix)
          xyb[(size_t)c * W * H + (size_t)(y0 + iy) * W + x0 + ix] +=
              kChannelDequant[c] * smp[(c * ys + iy) * xs + ix];
  }
  return ORC_OK;
}

/* ======================================================================= */
/* Dots (K.2)                                                              */
/* ======================================================================= */

/* K.2.1 LinDequant. */
static double lin_dequant(double x, double lo, double hi, double levels) {
  return (hi - lo) / levels * (x + 0.5) + lo;
}

/* K.2: n quantized dots (C.4.5), 10 integers each: x, y (times 5), sigma_x,
 * sigma_y, angle, sign_intensity, intensity[3], is_circle; each dequantized
 * (K.2.1) and added as a Gaussian over the 5 x 5 samples around
 * (floor(x), floor(y)) (K.2.2), in place.  Readings: kColourQuant, which the
 * draft never gives, is p->dot_colour_quant; a set sign bit negates its
 * channel's intensity (the printed assignment leaves it as it is); samples
 * of the window outside the frame are skipped. */
int orc_dots(const orc_params* p, const int32_t* dots, int32_t n, double* xyb) {
  const int32_t W = p->xsize, H = p->ysize;
  const double kPi = 3.14159265358979323846;
  for (int32_t k = 0; k < n; ++k) {
    const int32_t* q = dots + 10 * k;
    const double ex = q[0] / 5.0, ey = q[1] / 5.0;
    double angle, sx, sy;
    if (q[9]) {
      angle = 0.0;
      sx = sy = lin_dequant(q[2], 0.1, 3.1, 16);
    } else {
      angle = lin_dequant(q[4], 0.0, kPi, 8);
      sx = lin_dequant(q[2], 0.1, 3.1, 16);
      sy = lin_dequant(q[3], 0.1, 3.1, 16);
    }
    const double vx = sx * sx, vy = sy * sy;
    double inten[3];
    for (int c = 0; c < 3; ++c) {
      inten[c] = p->dot_colour_quant[c] * (q[6 + c] + 0.5);
      if (q[5] & (1 << c)) inten[c] = -inten[c];
    }
    inten[2] += 0.935669 * inten[1];
    const int32_t fx = (int32_t)floor(ex), fy = (int32_t)floor(ey);
    const double ca = cos(angle), sa = sin(angle);
    for (int32_t iy = fy - 2; iy <= fy + 2; ++iy)
      for (int32_t ix = fx - 2; ix <= fx + 2; ++ix) {
        if (ix < 0 || iy < 0 || ix >= W || iy >= H) continue;
        const double rx = ca * (ix - ex) + sa * (iy - ey);
        const double ry = -sa * (ix - ex) + ca * (iy - ey);
        const double md = rx * rx / vx + ry * ry / vy;
        const double g = exp(-0.5 * md);
        for (int c = 0; c < 3; ++c) xyb[(size_t)c * W * H + (size_t)iy * W + ix] += inten[c] * g;
      }
  }
  return ORC_OK;
}

/* ======================================================================= */
/* Splines (K.4)                                                           */
/* ======================================================================= */

/* K.4 ContinuousIDCT of one channel's 32 coefficients at t: DCTScale(k) is
 * D(32, k) of I.2.6.1 times 1/(4 sqrt 2) for k = 0, times 1/4 otherwise. */
double orc_spline_idct(const float* dct, double t) {
  const double kPi = 3.14159265358979323846;
  double s = 0.0;
  for (int k = 0; k < 32; ++k) {
    const double scale = orc_scale_D(32, k) * (k == 0 ? 1.0 / (4.0 * sqrt(2.0)) : 0.25);
    s += scale * dct[k] * cos(k * (kPi / 32.0) * (t + 0.5));
  }
  return s;
}

/* K.4 step 1: the sequence C sampling the centripetal Catmull-Rom curve
 * through the n control points pts[2n] (x, y): one control point alone, else
 * the control points extended by a mirrored point at each end, and for every
 * window of four consecutive points its second point followed by the curve
 * at 15 parameters strictly between the second and third (steps of one 16th
 * of that parameter interval), then the last control point.  cx, cy: room
 * for 16 (n - 1) + 1 points.  Returns the number of points, or -1 when two
 * consecutive control points coincide (a zero parameter interval). */
int32_t orc_spline_curve(const int32_t* pts, int32_t n, double* cx, double* cy) {
  if (n < 1) return -1;
  cx[0] = pts[0];
  cy[0] = pts[1];
  if (n == 1) return 1;
  for (int32_t i = 0; i + 1 < n; ++i)
    if (pts[2 * i] == pts[2 * i + 2] && pts[2 * i + 1] == pts[2 * i + 3]) return -1;
  /* E: Mirror(first, second), the control points, Mirror(last, second-to-last) */
  double* ex = (double*)malloc(sizeof(double) * (n + 2));
  double* ey = (double*)malloc(sizeof(double) * (n + 2));
  if (!ex || !ey) { free(ex); free(ey); return -1; }
  ex[0] = 2.0 * pts[0] - pts[2];
  ey[0] = 2.0 * pts[1] - pts[3];
  for (int32_t i = 0; i < n; ++i) { ex[i + 1] = pts[2 * i]; ey[i + 1] = pts[2 * i + 1]; }
  ex[n + 1] = 2.0 * pts[2 * n - 2] - pts[2 * n - 4];
  ey[n + 1] = 2.0 * pts[2 * n - 1] - pts[2 * n - 3];
  int32_t m = 0;
  for (int32_t w = 0; w + 3 < n + 2; ++w) {
    const double* px = ex + w;
    const double* py = ey + w;
    cx[m] = px[1];
    cy[m] = py[1];
    ++m;
    double tk[4];
    tk[0] = 0.0;
    for (int k = 1; k < 4; ++k) {
      const double dx = px[k] - px[k - 1], dy = py[k] - py[k - 1];
      tk[k] = tk[k - 1] + pow(dx * dx + dy * dy, 0.25);
    }
    for (int step = 1; step < 16; ++step) {
      const double t = tk[1] + step * (tk[2] - tk[1]) / 16.0;
      double ax[3], ay[3], bx[2], by[2];
      for (int k = 0; k < 3; ++k) {
        const double f = (t - tk[k]) / (tk[k + 1] - tk[k]);
        ax[k] = px[k] + f * (px[k + 1] - px[k]);
        ay[k] = py[k] + f * (py[k + 1] - py[k]);
      }
      for (int k = 0; k < 2; ++k) {
        const double f = (t - tk[k]) / (tk[k + 2] - tk[k]);
        bx[k] = ax[k] + f * (ax[k + 1] - ax[k]);
        by[k] = ay[k] + f * (ay[k + 1] - ay[k]);
      }
      const double f = (t - tk[1]) / (tk[2] - tk[1]);
      cx[m] = bx[0] + f * (bx[1] - bx[0]);
      cy[m] = by[0] + f * (by[1] - by[0]);
      ++m;
    }
  }
  cx[m] = ex[n];
  cy[m] = ey[n];
  ++m;
  free(ex);
  free(ey);
  return m;
}

/* K.4 step 2 to 3: the points P along the polyline through C (m points) at
 * arc lengths 0, 1, 2, ..., then the last point of C if the walk did not end
 * on it.  Writes up to cap points (x, y, arc position l, distance d from the
 * previous point, 1 for the first) and returns their number; *L_out: the
 * polyline's length.  Zero-length pieces of the polyline are passed over. */
int32_t orc_spline_walk(const double* cx, const double* cy, int32_t m, double* P, int32_t cap,
                        double* L_out) {
  double L = 0.0;
  for (int32_t i = 0; i + 1 < m; ++i) L += hypot(cx[i + 1] - cx[i], cy[i + 1] - cy[i]);
  *L_out = L;
  int32_t np = 0;
  if (np < cap) { P[0] = cx[0]; P[1] = cy[0]; P[2] = 0.0; P[3] = 1.0; }
  np = 1;
  double next = 1.0, arc = 0.0;
  for (int32_t i = 0; i + 1 < m; ++i) {
    const double len = hypot(cx[i + 1] - cx[i], cy[i + 1] - cy[i]);
    if (len == 0.0) continue;
    while (next <= arc + len) {
      const double f = (next - arc) / len;
      if (np < cap) {
        double* q = P + 4 * np;
        q[0] = cx[i] + f * (cx[i + 1] - cx[i]);
        q[1] = cy[i] + f * (cy[i + 1] - cy[i]);
        q[2] = next;
        q[3] = 1.0;
      }
      ++np;
      next += 1.0;
    }
    arc += len;
  }
  /* the last element of C unless the walk ended exactly on it */
  const double last = next - 1.0;
  if (m > 1 && last < L) {
    if (np < cap) {
      double* q = P + 4 * np;
      q[0] = cx[m - 1];
      q[1] = cy[m - 1];
      q[2] = L;
      q[3] = L - last;
    }
    ++np;
  }
  return np;
}

/* K.4: n splines added in place after the dots.  offsets[n + 1]: the
 * control points of spline s are pts[2 offsets[s] .. 2 offsets[s + 1]), as
 * (x, y); dct[n][4][32]: the dequantized and recorrelated DCT32 coefficients
 * of X, Y, B and sigma along the arc length.  Each point p of P (position l,
 * distance d) takes value = ContinuousIDCT(dct, 31 l / L) per channel and
 * adds, to every pixel (x, y) of the frame whose squared distance from p is
 * at most -2 sigma^2 log(0.1), value d sigma / 4 times the product of the
 * two differences of erf over the pixel's extent [x - 0.5, x + 0.5] (and the
 * same in y), each divided by sqrt(2) sigma.  Readings: "within r of p"
 * compares the squared distance with r (the Gaussian's tenth-of-peak
 * contour); steps of exactly one 16th of the parameter interval; a spline of
 * zero length (one control point) evaluates its values at t = 0; a point
 * whose sigma is not positive adds nothing.  near (may be NULL): [H][W],
 * set where a point's squared distance lies within 1e-9 of that bound,
 * relative (binary64 rounding can decide those pixels either way).  Returns
 * ORC_E_PARAM if a spline has no control points or two consecutive equal
 * ones. */
int orc_splines(const orc_params* p, const int32_t* offsets, int32_t n, const int32_t* pts,
                const float* dct, double* xyb, uint8_t* near) {
  const int32_t W = p->xsize, H = p->ysize;
  const size_t plane = (size_t)W * H;
  const double kLog01 = log(0.1);
  for (int32_t s = 0; s < n; ++s) {
    const int32_t nc = offsets[s + 1] - offsets[s];
    if (nc < 1) return ORC_E_PARAM;
    for (int32_t i = 0; i + 1 < nc; ++i) {
      const int32_t* q = pts + 2 * (offsets[s] + i);
      if (q[0] == q[2] && q[1] == q[3]) return ORC_E_PARAM;
    }
  }
  for (int32_t s = 0; s < n; ++s) {
    const int32_t nc = offsets[s + 1] - offsets[s];
    const int32_t cap_c = 16 * (nc - 1) + 1;
    double* cx = (double*)malloc(sizeof(double) * cap_c);
    double* cy = (double*)malloc(sizeof(double) * cap_c);
    if (!cx || !cy) { free(cx); free(cy); return ORC_E_SIZE; }
    const int32_t m = orc_spline_curve(pts + 2 * offsets[s], nc, cx, cy);
    double L;
    const int32_t np = orc_spline_walk(cx, cy, m, NULL, 0, &L);
    double* P = (double*)malloc(sizeof(double) * 4 * np);
    if (!P) { free(cx); free(cy); return ORC_E_SIZE; }
    orc_spline_walk(cx, cy, m, P, np, &L);
    const float* sd = dct + (size_t)s * 128;
    for (int32_t j = 0; j < np; ++j) {
      const double px = P[4 * j], py = P[4 * j + 1], l = P[4 * j + 2], d = P[4 * j + 3];
      const double t = L > 0.0 ? 31.0 * l / L : 0.0;
      double v[3];
      for (int c = 0; c < 3; ++c) v[c] = orc_spline_idct(sd + 32 * c, t);
      const double sigma = orc_spline_idct(sd + 96, t);
      if (!(sigma > 0.0)) continue;
      const double r2 = -2.0 * sigma * sigma * kLog01;
      const double r = sqrt(r2);
      const double s2s = sqrt(2.0) * sigma;
      const int32_t x0 = (int32_t)fmax(0.0, floor(px - r)), x1 = (int32_t)fmin(W - 1.0, ceil(px + r));
      const int32_t y0 = (int32_t)fmax(0.0, floor(py - r)), y1 = (int32_t)fmin(H - 1.0, ceil(py + r));
      for (int32_t y = y0; y <= y1; ++y)
        for (int32_t x = x0; x <= x1; ++x) {
          const double dx = px - x, dy = py - y;
          const double dd = dx * dx + dy * dy;
          if (near && fabs(dd - r2) <= 1e-9 * r2) near[(size_t)y * W + x] = 1;
          if (dd > r2) continue;
          const double g = (erf((dx + 0.5) / s2s) - erf((dx - 0.5) / s2s)) *
                           (erf((dy + 0.5) / s2s) - erf((dy - 0.5) / s2s));
          for (int c = 0; c < 3; ++c)
            xyb[c * plane + (size_t)y * W + x] += v[c] * d * sigma / 4.0 * g;
        }
    }
    free(P);
    free(cx);
    free(cy);
  }
  return ORC_OK;
}

/* ======================================================================= */
/* Noise (K.5)                                                             */
/* ======================================================================= */

/* K.5.2: the draft's SplitMix64 mixing function of a 64-bit state. */
uint64_t orc_splitmix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}

/* K.5.2: one XorShift128+ step of one generator on its state (s0, s1), in
 * place; returns batch[i].  Reading: the printed step updates s1 only; a
 * XorShift128+ step also moves the old second word into the first place, so
 * after it s1 takes the old s0 and s0 the updated value (without the
 * exchange s0 would never change). */
uint64_t orc_noise_step(uint64_t* s0, uint64_t* s1) {
  /* the printed step, then the two state words change places (s1 the first
   * word, s0 the second) */
  const uint64_t t = *s0;
  *s1 ^= *s1 << 23;
  const uint64_t b = *s1 + *s0;
  *s1 ^= *s0 ^ (*s1 >> 18) ^ (*s0 >> 5);
  *s0 = *s1;
  *s1 = t;
  return b;
}

/* K.5.2: the three pseudorandom channels RR, RG, RB of the group whose
 * top-left pixel is (x0, y0), gw x gh samples each: eight XorShift128+
 * generators seeded from (y0 << 32) + x0 through SplitMix64; per row and per
 * segment of up to 16 samples one step of all eight gives sixteen 32-bit
 * words, sample j of the segment being the binary32 with exponent 0 and the
 * top 23 bits of word j as mantissa, minus 1.  Channels, rows and segments
 * follow in that order from one generator state.  out: [3][gh][gw]. */
void orc_noise_channels(int32_t gw, int32_t gh, int32_t x0, int32_t y0, float* out) {
  uint64_t s0[8], s1[8];
  const uint64_t seed = ((uint64_t)(uint32_t)y0 << 32) + (uint64_t)(uint32_t)x0;
  s0[0] = orc_splitmix64(seed + 0x9E3779B97F4A7C15ull);
  s1[0] = orc_splitmix64(s0[0]);
  for (int i = 1; i < 8; ++i) {
    s0[i] = orc_splitmix64(s1[i - 1]);
    s1[i] = orc_splitmix64(s0[i]);
  }
  for (int c = 0; c < 3; ++c)
    for (int32_t y = 0; y < gh; ++y)
      for (int32_t x = 0; x < gw; x += 16) {
        uint32_t bits[16];
        for (int i = 0; i < 8; ++i) {
          const uint64_t b = orc_noise_step(&s0[i], &s1[i]);
          bits[2 * i] = (uint32_t)b;
          bits[2 * i + 1] = (uint32_t)(b >> 32);
        }
        for (int j = 0; j < 16 && x + j < gw; ++j) {
          const uint32_t u = (bits[j] >> 9) | 0x3F800000u;
          float f;
          memcpy(&f, &u, sizeof(f));
          out[((size_t)c * gh + y) * gw + x + j] = f - 1.0f;
        }
      }
}

/* K.5: noise over a cropped XYB frame (after Gaborish), per group of 256 x 256
 * pixels (6.2): the three channels of K.5.2, each convolved with the 5x5
 * kernel of 1 at distance 2 up, down, left and right and -4 at the centre
 * (6.5 mirroring at the group's size), times 0.22, give A_R, A_G, A_B; the
 * strengths S_R, S_G from the LUT at 14 (Y + X) and 14 (Y - X) (integer part
 * clamped to [0, 14], linear interpolation with the fractional part, result
 * clamped to [0, 1]); N_R = (0.01 A_R + 0.99 A_B) S_R and
 * N_G = (0.01 A_G + 0.99 A_B) S_G are added: X += N_R - N_G,
 * Y += N_R + N_G, B += 0.935669 (N_R + N_G).  Readings: the channels are
 * generated at the group's size, and the 5x5 kernel mirrors at the group's
 * edges; the clamp of the integer part to [0, 14] bounds the scaled input
 * to [0, 15] before the split (the strength is the LUT interpolated on
 * [0, 15] and held at its end values outside; taking the fraction before the
 * clamp would make the strength jump from LUT[0] to LUT[1] where the input
 * crosses 0). */
int orc_noise(const orc_params* p, const double* in, double* out) {
  int st = check_params(p);
  if (st) return st;
  const int32_t W = p->xsize, H = p->ysize;
  const size_t plane = (size_t)W * H;
  memcpy(out, in, sizeof(double) * 3 * plane);
  float* ch = (float*)malloc(sizeof(float) * 3 * 256 * 256);
  if (!ch) return ORC_E_SIZE;
  for (int32_t y0 = 0; y0 < H; y0 += 256)
    for (int32_t x0 = 0; x0 < W; x0 += 256) {
      const int32_t gw = W - x0 < 256 ? W - x0 : 256, gh = H - y0 < 256 ? H - y0 : 256;
      orc_noise_channels(gw, gh, x0, y0, ch);
      for (int32_t y = 0; y < gh; ++y)
        for (int32_t x = 0; x < gw; ++x) {
          double A[3];
          for (int c = 0; c < 3; ++c) {
            const float* r = ch + (size_t)c * gh * gw;
#define R_AT(yy, xx) ((double)r[(size_t)mirror((yy), gh) * gw + mirror((xx), gw)])
            A[c] = 0.22 * (R_AT(y - 2, x) + R_AT(y, x - 2) + R_AT(y, x + 2) + R_AT(y + 2, x) -
                           4.0 * R_AT(y, x));
#undef R_AT
          }
          const size_t i = (size_t)(y0 + y) * W + x0 + x;
          const double X = in[i], Y = in[plane + i];
          double S[2];
          const double inp[2] = {Y + X, Y - X};
          for (int k = 0; k < 2; ++k) {
            double sc = inp[k] * 14.0;
            sc = sc < 0.0 ? 0.0 : sc > 15.0 ? 15.0 : sc;
            double in_int = floor(sc);
            if (in_int > 14.0) in_int = 14.0;
            const double in_frac = sc - in_int;
            const int ii = (int)in_int;
            double v = p->noise_lut[ii] * (1.0 - in_frac) + p->noise_lut[ii + 1] * in_frac;
            S[k] = v < 0.0 ? 0.0 : v > 1.0 ? 1.0 : v;
          }
          const double NR = 0.01 * A[0] * S[0] + 0.99 * A[2] * S[0];
          const double NG = 0.01 * A[1] * S[1] + 0.99 * A[2] * S[1];
          out[i] = X + NR - NG;
          out[plane + i] = Y + NR + NG;
          out[2 * plane + i] = in[2 * plane + i] + 0.935669 * (NR + NG);
        }
    }
  free(ch);
  return ORC_OK;
}

/* ======================================================================= */
/* Gaborish (J.4)                                                          */
/* ======================================================================= */

/* Reading: the weights are the loop-filter fields themselves; the printed
 * factor 10^-6 contradicts the field defaults (0.115..., 0.061...), which are
 * already fractions of the centre weight. */
int orc_gaborish(const orc_params* p, const double* in, double* out) {
  int st = check_params(p);
  if (st) return st;
  const int32_t W = p->xsize, H = p->ysize;
  const size_t plane = (size_t)W * H;
  for (int c = 0; c < 3; ++c) {
    const double norm = 1.0 + 4.0 * p->gab_w1[c] + 4.0 * p->gab_w2[c];
    double k[3][3];
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        int taxi = abs(dx) + abs(dy);
        double w = taxi == 0 ? 1.0 : (taxi == 1 ? p->gab_w1[c] : p->gab_w2[c]);
        k[dy + 1][dx + 1] = w / norm;
      }
#pragma omp parallel for
    for (int32_t y = 0; y < H; ++y)
      for (int32_t x = 0; x < W; ++x) {
        double acc = 0.0;
        for (int dy = -1; dy <= 1; ++dy)
          for (int dx = -1; dx <= 1; ++dx)
            acc += k[dy + 1][dx + 1] *
                   in[c * plane + (size_t)mirror(y + dy, H) * W + mirror(x + dx, W)];
        out[c * plane + (size_t)y * W + x] = acc;
      }
  }
  return ORC_OK;
}

/* ======================================================================= */
/* XYB -> RGB (L.2)                                                        */
/* ======================================================================= */

int orc_xyb_to_rgb(const orc_params* p, const double* xyb, double* rgb) {
  int st = check_params(p);
  if (st) return st;
  const size_t plane = (size_t)p->xsize * p->ysize;
  const double scale = p->target_nits_div50 * 50.0 / 250.0;
#pragma omp parallel for
  for (int64_t i = 0; i < (int64_t)plane; ++i) {
    double X = xyb[i], Y = xyb[plane + i], B = xyb[2 * plane + i];
    double g[3] = {Y + X, Y - X, B};
    double mix[3];
    for (int c = 0; c < 3; ++c) mix[c] = g[c] * g[c] * g[c] + p->opsin_bias[c];
    for (int r = 0; r < 3; ++r) {
      double v = 0.0;
      for (int c = 0; c < 3; ++c) v += p->opsin_inv[r * 3 + c] * mix[c];
      /* Divided by target_nits_div50 * 50 / 250, then by 255 for [0, 1]. */
      rgb[r * plane + i] = v / scale / 255.0;
    }
  }
  return ORC_OK;
}

/* Reading for 8- and 16-bit output: the sRGB transfer function
 * (IEC 61966-2-1) applied to the linear value clamped to [0, 1], then
 * Q_b(v) = floor(v * (2^b - 1) + 0.5). */
int orc_quantize_srgb(int32_t bits, int64_t n, const double* lin, uint16_t* out) {
  if (bits != 8 && bits != 16) return ORC_E_PARAM;
  const double maxv = (double)((1 << bits) - 1);
  for (int64_t i = 0; i < n; ++i) {
    double v = lin[i];
    v = v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
    double e = v <= 0.0031308 ? 12.92 * v : 1.055 * pow(v, 1.0 / 2.4) - 0.055;
    out[i] = (uint16_t)floor(e * maxv + 0.5);
  }
  return ORC_OK;
}

/* ======================================================================= */
/* JPEG1 direct rasterization (M.6)                                        */
/* ======================================================================= */

/* M.6.1 and M.6.2: one component of wib x hib blocks; qcoef int32
 * [8 hib][8 wib], coefficient index 8 u + v of block (bx, by) at row
 * 8 by + u, column 8 bx + v; quant[64] by the same index.  Each coefficient
 * is multiplied by its quantization step and I(8, u) I(8, v) (I.2.6.1), then
 * the block goes through IDCT_2D (I.2.2) with u the vertical and v the
 * horizontal frequency (the layout of JPEG1's natural coefficient order).
 * out: pixels [8 hib][8 wib].  The conditioning of M.6.1.1 is not applied
 * (it is driven by an optional side channel). */
int orc_jpeg1_component(const int32_t* qcoef, int32_t wib, int32_t hib, const int32_t* quant,
                        double* out) {
  if (wib < 1 || hib < 1) return ORC_E_SIZE;
  const int32_t W = 8 * wib;
  double T[64];
  orc_idct_matrix(8, T);
  for (int32_t by = 0; by < hib; ++by)
    for (int32_t bx = 0; bx < wib; ++bx) {
      double K[64], tmp[64];
      for (int u = 0; u < 8; ++u)
        for (int v = 0; v < 8; ++v)
          K[8 * u + v] = (double)qcoef[(size_t)(8 * by + u) * W + 8 * bx + v] * quant[8 * u + v] *
                         orc_scale_I(8, u) * orc_scale_I(8, v);
      /* columns (vertical frequency u), then rows (horizontal frequency v) */
      for (int y = 0; y < 8; ++y)
        for (int v = 0; v < 8; ++v) {
          double acc = 0.0;
          for (int u = 0; u < 8; ++u) acc += T[y * 8 + u] * K[8 * u + v];
          tmp[8 * y + v] = acc;
        }
      for (int y = 0; y < 8; ++y)
        for (int x = 0; x < 8; ++x) {
          double acc = 0.0;
          for (int v = 0; v < 8; ++v) acc += T[x * 8 + v] * tmp[8 * y + v];
          out[(size_t)(8 * by + y) * W + 8 * bx + x] = acc;
        }
    }
  return ORC_OK;
}

/* M.6.3: the side channel's block-gated Gaborish on one component's pixels
 * [8 hib][8 wib] (the output of M.6.2), in place.  code: the four decoded
 * bytes gab_weight1 * 1024, gab_weight2 * 1024, threshold * 16 and limit.
 * The smoothed plane is the J.4 convolution (centre 1, edge neighbours
 * gab_weight1, diagonal ones gab_weight2, normalized to sum 1) of the
 * pixels, mirrored (6.5) at the plane's edges; every 8 x 8 block takes the
 * smoothed values when fewer than `limit` of its 6 x 6 interior pixels
 * (offsets 1..6 both ways) differ from them by more than the threshold,
 * and keeps its own otherwise.  Reading: the plane is the component's
 * block-padded plane, as for the upsampling. */
int orc_jpeg1_gaborish(double* pix, int32_t wib, int32_t hib, const uint8_t* code) {
  if (wib < 1 || hib < 1) return ORC_E_SIZE;
  const int32_t W = 8 * wib, H = 8 * hib;
  const double w1 = code[0] / 1024.0, w2 = code[1] / 1024.0;
  const double thr = code[2] / 16.0;
  const int limit = code[3];
  const double norm = 1.0 + 4.0 * w1 + 4.0 * w2;
  double* sm = (double*)malloc(sizeof(double) * (size_t)W * H);
  if (!sm) return ORC_E_SIZE;
  for (int32_t y = 0; y < H; ++y)
    for (int32_t x = 0; x < W; ++x) {
      double acc = 0.0;
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int taxi = abs(dx) + abs(dy);
          const double w = taxi == 0 ? 1.0 : (taxi == 1 ? w1 : w2);
          acc += w / norm * pix[(size_t)mirror(y + dy, H) * W + mirror(x + dx, W)];
        }
      sm[(size_t)y * W + x] = acc;
    }
  for (int32_t by = 0; by < hib; ++by)
    for (int32_t bx = 0; bx < wib; ++bx) {
      int count = 0;
      for (int v = 1; v < 7; ++v)
        for (int u = 1; u < 7; ++u) {
          const size_t o = (size_t)(8 * by + v) * W + 8 * bx + u;
          if (fabs(pix[o] - sm[o]) > thr) ++count;
        }
      if (count < limit)
        for (int v = 0; v < 8; ++v)
          for (int u = 0; u < 8; ++u) {
            const size_t o = (size_t)(8 * by + v) * W + 8 * bx + u;
            pix[o] = sm[o];
          }
    }
  free(sm);
  return ORC_OK;
}

/* M.6.4: linear 2x upsampling of n samples with respect to pixel centres,
 * mirrored at both ends (index -1 reads index 1, index n reads n - 2):
 * out[2i] = 3/4 a[i] + 1/4 a[i - 1], out[2i + 1] = 3/4 a[i] + 1/4 a[i + 1],
 * with the given stride between samples (in and out). */
void orc_upsample2(const double* in, int32_t n, size_t stride_in, double* out,
                   size_t stride_out) {
  for (int32_t i = 0; i < n; ++i) {
    const int32_t l = i == 0 ? (n > 1 ? 1 : 0) : i - 1;
    const int32_t r = i == n - 1 ? (n > 1 ? n - 2 : 0) : i + 1;
    const double a = in[i * stride_in];
    out[(size_t)(2 * i) * stride_out] = 0.75 * a + 0.25 * in[l * stride_in];
    out[(size_t)(2 * i + 1) * stride_out] = 0.75 * a + 0.25 * in[r * stride_in];
  }
}

/* M.6.4 to M.6.6: three components (Y, Cb, Cr) of pixels [8 hib_c][8 wib_c]
 * with sampling factors hs[c], vs[c] in {1, 2} (the largest being the
 * luma's), upsampled where a component's factor is below the largest
 * (horizontally first), transformed to RGB by M.6.5 and cropped to xsize x
 * ysize.  Readings: a component is upsampled over its whole block-padded
 * plane, mirrored at that plane's edges, before the crop; one component
 * gives grey (R = G = B = Y + 128).  rgb: [3][ysize][xsize]. */
int orc_jpeg1_rasterize(int32_t ncomp, const double* const pix[3], const int32_t* wib,
                        const int32_t* hib, const int32_t* hs, const int32_t* vs, int32_t xsize,
                        int32_t ysize, double* rgb) {
  if (ncomp != 1 && ncomp != 3) return ORC_E_PARAM;
  if (xsize < 1 || ysize < 1) return ORC_E_SIZE;
  int32_t hmax = 1, vmax = 1;
  for (int c = 0; c < ncomp; ++c) {
    if (hs[c] < 1 || hs[c] > 2 || vs[c] < 1 || vs[c] > 2) return ORC_E_PARAM;
    if (hs[c] > hmax) hmax = hs[c];
    if (vs[c] > vmax) vmax = vs[c];
  }
  double* full[3] = {NULL, NULL, NULL};
  int st = ORC_OK;
  for (int c = 0; c < ncomp && !st; ++c) {
    const int32_t w = 8 * wib[c], h = 8 * hib[c];
    const int32_t fx = hmax / hs[c], fy = vmax / vs[c];
    if (w * fx < xsize || h * fy < ysize) { st = ORC_E_SIZE; break; }
    double* hor = (double*)malloc(sizeof(double) * (size_t)w * fx * h);
    full[c] = (double*)malloc(sizeof(double) * (size_t)w * fx * h * fy);
    if (!hor || !full[c]) { free(hor); st = ORC_E_SIZE; break; }
    for (int32_t y = 0; y < h; ++y) {
      if (fx == 2) orc_upsample2(pix[c] + (size_t)y * w, w, 1, hor + (size_t)y * 2 * w, 1);
      else memcpy(hor + (size_t)y * w, pix[c] + (size_t)y * w, sizeof(double) * w);
    }
    const int32_t W2 = w * fx;
    for (int32_t x = 0; x < W2; ++x) {
      if (fy == 2) orc_upsample2(hor + x, h, W2, full[c] + x, W2);
      else for (int32_t y = 0; y < h; ++y) full[c][(size_t)y * W2 + x] = hor[(size_t)y * W2 + x];
    }
    free(hor);
  }
  if (!st) {
    const size_t plane = (size_t)xsize * ysize;
    for (int32_t y = 0; y < ysize; ++y)
      for (int32_t x = 0; x < xsize; ++x) {
        const size_t o = (size_t)y * xsize + x;
        const double Y = full[0][(size_t)y * 8 * wib[0] * (hmax / hs[0]) + x];
        if (ncomp == 1) {
          rgb[o] = rgb[plane + o] = rgb[2 * plane + o] = Y + 128.0;
          continue;
        }
        const double Cb = full[1][(size_t)y * 8 * wib[1] * (hmax / hs[1]) + x];
        const double Cr = full[2][(size_t)y * 8 * wib[2] * (hmax / hs[2]) + x];
        rgb[o] = 1.402 * Cr + (Y + 128.0);
        rgb[plane + o] = -0.71414 * Cr - 0.34414 * Cb + (Y + 128.0);
        rgb[2 * plane + o] = 1.772 * Cb + (Y + 128.0);
      }
  }
  for (int c = 0; c < 3; ++c) free(full[c]);
  return st;
}

/* ======================================================================= */
/* Whole path (9.7-9.13)                                                   */
/* ======================================================================= */

int orc_decode(const orc_params* p, const int32_t* const ac[3], const int32_t* const dc[3],
               const uint8_t* strategy, const uint8_t* qf_minus_1, const uint8_t* sharpness,
               const float* cfl_kx, const float* cfl_kb, double* rgb) {
  return orc_decode_features(p, ac, dc, strategy, qf_minus_1, sharpness, cfl_kx, cfl_kb, NULL, 0,
                             NULL, NULL, 0, NULL, 0, NULL, NULL, rgb);
}

int orc_decode_features(const orc_params* p, const int32_t* const ac[3],
                        const int32_t* const dc[3], const uint8_t* strategy,
                        const uint8_t* qf_minus_1, const uint8_t* sharpness, const float* cfl_kx,
                        const float* cfl_kb, const int32_t* patch_place, int32_t n_patches,
                        const int32_t* patch_samples, const int32_t* dots, int32_t n_dots,
                        const int32_t* spline_offsets, int32_t n_splines,
                        const int32_t* spline_points, const float* spline_dct, double* rgb) {
  int st = check_params(p);
  if (st) return st;
  const size_t n = 3 * (size_t)p->xsize * p->ysize;
  double* a = (double*)malloc(sizeof(double) * n);
  double* b = (double*)malloc(sizeof(double) * n);
  if (!a || !b) { free(a); free(b); return ORC_E_SIZE; }
  st = orc_reconstruct(p, ac, dc, strategy, qf_minus_1, cfl_kx, cfl_kb, a);
  double* r = NULL;
  if (!st && p->qco && p->epf_iters > 0) {
    r = (double*)malloc(sizeof(double) * n);
    if (!r) st = ORC_E_SIZE;
    else memcpy(r, a, sizeof(double) * n);
  }
  for (int it = 0; !st && it < p->epf_iters; ++it) {
    st = orc_epf_pass(p, strategy, qf_minus_1, sharpness, a, b, NULL, NULL);
    double* t = a; a = b; b = t;
  }
  /* J.1: the constraint follows the filter passes, against their input */
  if (!st && r) {
    st = orc_qco(p, strategy, qf_minus_1, r, a, b);
    double* t = a; a = b; b = t;
  }
  free(r);
  /* K.1: patches between adaptive reconstruction and Gaborish */
  if (!st && n_patches > 0) st = orc_patches(p, patch_place, n_patches, patch_samples, a);
  if (!st && p->gab) {
    st = orc_gaborish(p, a, b);
    double* t = a; a = b; b = t;
  }
  /* K.1: dots, then noise, after Gaborish */
  if (!st && n_dots > 0) st = orc_dots(p, dots, n_dots, a);
  /* K.4: splines after the dots */
  if (!st && n_splines > 0)
    st = orc_splines(p, spline_offsets, n_splines, spline_points, spline_dct, a, NULL);
  if (!st && p->noise) {
    st = orc_noise(p, a, b);
    double* t = a; a = b; b = t;
  }
  if (!st) st = orc_xyb_to_rgb(p, a, rgb);
  free(a);
  free(b);
  return st;
}
