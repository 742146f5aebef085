/*
 * jxlr.h -- JPEG XL VarDCT pixel reconstruction on MI355X (gfx950), C ABI.
 *
 * Implements the data-parallel part of the VarDCT decoding process of the
 * JPEG XL Committee Draft (ISO/IEC 18181 CD, 2019-08-05): from entropy-decoded
 * quantized coefficients to RGB samples, in the draft's stage order
 *   F.2/F.3 dequantization -> Annex G chroma from luma -> I.2.7 LLF from DC
 *   -> I.2.4 inverse transform selected by DctSelect (C.5.4)
 *   -> J.2 edge-preserving filter (0..n passes) -> J.4 Gaborish
 *   -> L.2 XYB to RGB (and optional sRGB 8/16-bit encoding).
 * Entropy decoding (Annex D) and bitstream parsing are not part of it: the
 * caller passes decoded header fields and sample planes.
 *
 * Memory: every plane pointer in jxlr_frame_io and every workspace/debug
 * pointer is a DEVICE pointer on the context's device, owned by the caller.
 * The library never allocates or frees inside a decode call; it allocates only
 * its constant tables in jxlr_create and frees them in jxlr_destroy.
 *
 * Ordering: launches are asynchronous on the given stream (NULL = the null
 * stream) and ordered with other work on it.  Parameter and size errors are
 * reported synchronously, before anything is enqueued.  A DctSelect map that
 * is ill-formed (C.5.4) is detected on the device: the affected 32 x 32 regions
 * are written as zero and a sticky flag is set that jxlr_get_device_status
 * reports (an ill-formed patch placement, K.3, sets it as well);
 * jxlr_validate_maps_host checks the map rules on the host first.
 * On any error no output content is guaranteed.
 *
 * Threading: a context may be used from several host threads and streams at
 * once, provided each concurrent call has its own workspace and outputs; the
 * sticky device-validation flag is one per context (jxlr_get_device_status).
 */
#ifndef JXLR_H
#define JXLR_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  JXLR_OK = 0,
  JXLR_E_NULL = 1,        /* a required pointer is NULL */
  JXLR_E_SIZE = 2,        /* xsize/ysize zero or above JXLR_MAX_DIM, or a stride too small */
  JXLR_E_STRATEGY = 3,    /* DctSelect value not in the C.5.4 table or not supported */
  JXLR_E_ALIGN = 4,       /* varblock not naturally aligned, out of bounds or overlapping (C.5.4) */
  JXLR_E_QUANT = 5,       /* quant field not uniform within a varblock (C.5.5) */
  JXLR_E_DEQUANT = 6,     /* dequantization matrix entry not positive and finite (C.6.1) */
  JXLR_E_PARAM = 7,       /* frame parameter out of range (see jxlr_frame_params) */
  JXLR_E_WORKSPACE = 8,   /* workspace smaller than jxlr_workspace_bytes */
  JXLR_E_HIP = 9,         /* a HIP runtime call failed */
  JXLR_E_DEVICE_VALIDATION = 10 /* sticky: the device found an ill-formed DctSelect map */
} jxlr_status;

/* Transform types; numbering of the C.5.4 table.  This library reconstructs
 * all fifteen (inverse transforms of I.2.4.1-I.2.4.7); values from 15 up are
 * rejected with JXLR_E_STRATEGY.  "DCT N x M" covers bxsize = max(8, N) by
 * bysize = max(8, M) pixels (I.2.5): the first number is the width; DCT4X8,
 * DCT8X4 and AFV cover 8 x 8. */
typedef enum {
  JXLR_DCT8 = 0, JXLR_IDENTITY = 1, JXLR_DCT2 = 2, JXLR_DCT4 = 3, JXLR_DCT16 = 4,
  JXLR_DCT32 = 5, JXLR_DCT16X8 = 6, JXLR_DCT8X16 = 7, JXLR_DCT32X8 = 8,
  JXLR_DCT8X32 = 9, JXLR_DCT32X16 = 10, JXLR_DCT16X32 = 11, JXLR_DCT4X8 = 12,
  JXLR_DCT8X4 = 13, JXLR_AFV = 14
} jxlr_strategy;

/* Output sample formats.  F32: linear RGB of L.2 divided by 255 ("[0,1]-scaled",
 * not clamped).  U8/U16: the sRGB transfer function (IEC 61966-2-1) applied to
 * the [0,1]-scaled value clamped to [0, 1], then floor(v * (2^b - 1) + 0.5). */
typedef enum { JXLR_OUT_F32 = 0, JXLR_OUT_U8_SRGB = 1, JXLR_OUT_U16_SRGB = 2 } jxlr_out_format;

#define JXLR_MAX_DIM 65536u

/* Encoding modes of a dequantization matrix (C.6.1). */
typedef enum {
  JXLR_DQ_LIBRARY = 0, JXLR_DQ_IDENTITY = 1, JXLR_DQ_DCT2 = 2, JXLR_DQ_DCT4 = 3,
  JXLR_DQ_DCT4X8 = 4, JXLR_DQ_AFV = 5, JXLR_DQ_DCT = 6, JXLR_DQ_COPY = 7
} jxlr_dequant_mode;

/* One dequantization matrix's encoding (C.6.1), already read from the
 * stream (the F16 parameters as their values).  Fields a mode does not read
 * are ignored.  Per channel X, Y, B:
 *   LIBRARY   the C.6.1.1 default encoding of this matrix;
 *   IDENTITY  params[c][0..2];             DCT2  params[c][0..5];
 *   DCT4      params[c][0..1] and the bands;
 *   DCT4X8    params[c][0] (dct4x8multipliers) and the bands;
 *   AFV       params[c][0..1] (dct4multipliers), afv_weights[c][0..7];
 *   DCT       the bands;
 *   COPY      the encoding of matrix copy_from, which must be smaller than
 *             this matrix's index (evaluated for this matrix's type).
 * Bands: num_bands distance bands dist_bands[c][0..num_bands-1], 2..17, and
 * num_ecc_bands eccentricity bands ecc_bands[c][0..num_ecc_bands-1], 1..8.
 * IDENTITY, DCT2, DCT4, DCT4X8 and AFV define 64-entry matrices only (types
 * DCT8, IDENTITY, DCT2, DCT4, DCT4X8, DCT8X4, AFV); DCT4X8 is transposed for
 * DCT8X4. */
typedef struct {
  int32_t mode;
  int32_t copy_from;
  int32_t num_bands;
  int32_t num_ecc_bands;
  double  dist_bands[3][17];
  double  ecc_bands[3][8];
  double  params[3][6];
  double  afv_weights[3][8];
} jxlr_dequant_encoding;

/* Decoded frame-header fields.  Channel order X, Y, B.  jxlr_params_default
 * fills the draft's defaults. */
typedef struct {
  uint32_t xsize, ysize;       /* frame size in pixels, 1..JXLR_MAX_DIM (A.4.2, 6.2) */
  uint32_t global_scale;       /* global_scale_minus_1 + 1, 1..65536 (C.4.2) */
  float    dc_mul[3];          /* mX_DC, mY_DC, mB_DC of C.4.1, already divided by
                                  global_scale * (quant_dc_minus_1 + 1) */
  int32_t  extra_levels[3];    /* extra_levels_xyb of C.5.2, 0..3 */
  float    kx_dc, kb_dc;       /* DC chroma-from-luma factors as kX, kB (C.4.3, Annex G) */
  int32_t  gab;                /* loop_filter.gab: apply Gaborish (C.10, J.4) */
  float    gab_w1[3], gab_w2[3]; /* Gaborish edge and corner weights per channel (C.10) */
  int32_t  epf_iters;          /* edge-preserving filter passes, 0..3; 0 = loop_filter.epf off */
  float    epf_weight_min;     /* C.10; at most 1 */
  float    epf_scale[3];       /* C.10 */
  float    epf_sharp_lut[8];   /* C.10 */
  float    epf_range_max, epf_range_mul, epf_quant_mul; /* C.10 */
  int32_t  epf_sigma_max;      /* C.10, 0..672 */
  int32_t  epf_sigma_shift;    /* kSigmaShift of J.2.4 (undefined by the draft), 0..8 */
  float    opsin_inv[9];       /* inverse opsin absorbance matrix, row-major (L.2, C.4.9) */
  float    opsin_bias[3];      /* opsin biases (L.2, C.4.9) */
  int32_t  target_nits_div50;  /* ImageMetadata (A.4.5), >= 1 */
  int32_t  out_format;         /* jxlr_out_format */
  /* Inverse-transform arithmetic.  0: binary32 throughout (the plain form).
   * 1: split precision, for every 32x32 region tiled by varblocks of one
   * DCT type (DCT8, DCT16, DCT32 and the rectangular DCTs): the column and
   * the row pass of the high-frequency coefficients are matrix products on
   * the matrix cores, their operands scaled by a power of two per wave and
   * split into binary16 high and low parts, hi*hi + hi*lo + lo*hi
   * accumulated in binary32; each varblock's LLF corner is transformed in
   * binary32 beside them; other regions use the plain form. */
  int32_t  idct_split;
  /* Adaptive DC smoothing of F.2 (1) or not (0, the default; the draft's
   * kSkipAdaptiveDCSmoothing case): each dequantized DC sample away from the
   * frame's first and last block row and column becomes the 3x3 weighted
   * average of its neighbourhood when that lies within 0.5 dcq of it, dcq =
   * the sample's DcQuantField (C.5.2; io->dc_quant, or dc_mul[c] /
   * 2^extra_levels[c] without it).  Applied before the DC chroma from luma
   * and the LLF computation. */
  int32_t  dc_smoothing;
  /* Quantization constraint of J.3 (loop_filter.qco, default 0), applied once
   * after the last EPF pass (none without EPF): per varblock and channel the
   * residual of the filter passes is transformed to coefficients, each
   * clamped to +-qco_interval_mul quantization steps (dequantization weight
   * times AcMul; for the LLF corner, each of its DC samples to
   * +-qco_interval_mul times that sample's DcQuantField), and transformed
   * back. */
  int32_t  qco;
  float    qco_interval_mul;  /* C.10 default 0.5; finite, >= 0 */
  /* AC prediction of Annex H (1) or not (0, the default; the draft's
   * kSkipPredictLF case): per group of 256x256 samples an image of 2x2 cells
   * per block (I.2.6 at N = 4 of each varblock's LLF, a border from the DC
   * ring around the group, mirrored at the frame edge), adaptively smoothed
   * (0.12 / 0.2 / 0.02 weights, accepted within 1.7 dc_mul[c], the DC
   * multiplier of C.4.1 itself), then I.2.7 at N = 4 gives each varblock's top 2cy x 2cx
   * coefficients, which are added (LLF corner excepted) after the chroma
   * from luma.  Needs io->ac_pred for jxlr_reconstruct (filled by
   * jxlr_ac_prediction); jxlr_decode and the batch functions manage it. */
  int32_t  ac_prediction;
  /* Noise of K.5 (1; kNoise) or not (0, the default), after Gaborish: per
   * 256x256 group three pseudorandom channels (K.5.2; SplitMix64-seeded
   * XorShift128+, made by jxlr_noise_channels), their 5x5 Laplacian times
   * 0.22, modulated by the strengths the LUT gives at 14 (Y + X) and
   * 14 (Y - X).  Needs io->noise_raw for jxlr_finish; jxlr_decode and the
   * batch functions manage it. */
  int32_t  noise;
  float    noise_lut[16];     /* C.4.8: u(10) / 1024 each; finite */
  /* Patches of K.3: the number of placements in io->patch_place (0: none),
   * added between the EPF passes (and the quantization constraint) and
   * Gaborish. */
  int32_t  num_patches;
  /* Dots of K.2: the number of quantized dots in io->dots (0: none), added
   * after Gaborish (and before the noise); with dots, jxlr_finish skips its
   * Gaborish and the caller runs jxlr_gaborish then jxlr_dots before it
   * (jxlr_decode does).  dot_colour_quant: the draft's kColourQuant, which it
   * does not give (finite). */
  int32_t  num_dots;
  float    dot_colour_quant[3];
  /* Splines of K.4: the number of splines in io (0: none), rendered after
   * the dots (and before the noise); like dots they make Gaborish a pass of
   * its own.  num_spline_points: the control points of all of them (at
   * least one each, at most 2^22 in all); it sizes the curve scratch. */
  int32_t  num_splines;
  int32_t  num_spline_points;
  /* The finish fused into the stage before it, for a frame that qualifies
   * (no patches, dots, splines or noise, no quantization constraint after
   * EPF passes): into the reconstruction (jxlr_reconstruct_finish) when the
   * frame has no EPF pass, else into the last EPF pass (jxlr_epf_finish).
   * 0 (the default) lets the library choose the reconstruction's tiles per
   * run, 1..4 sets them, -1 keeps the stages apart (jxlr_decode then stores
   * the XYB frame in its workspace).  The output does not depend on it. */
  int32_t  fuse;
} jxlr_frame_params;

/* Input and output planes of one frame.  With Wb = ceil(xsize/8),
 * Hb = ceil(ysize/8), Wt = ceil(xsize/64), Ht = ceil(ysize/64):
 *   ac[c]      int32 [8*Hb rows][8*Wb], row stride ac_stride (elements):
 *              quantized AC coefficients; coefficient (x, y) of the varblock
 *              with top-left block (bx0, by0) sits at (8*bx0 + x, 8*by0 + y);
 *              the varblock's LLF corner (x < bx/8, y < by/8) is ignored (F.2)
 *   dc[c]      int32 [Hb][Wb], stride dc_stride: quantized DC (C.5.2, F.2)
 *   strategy   uint8 [Hb][Wb], stride map_stride: DctSelect (C.5.4); only the
 *              entry at each varblock's top-left block is read
 *   qf_minus_1 uint8 [Hb][Wb], stride map_stride: quant field value dv of
 *              C.5.5 (AcMul = 65536 / (global_scale * (1 + dv))); uniform per
 *              varblock
 *   sharpness  uint8 [Hb][Wb], stride map_stride: C.5.6, 0..7 (read only
 *              when epf_iters > 0)
 *   cfl_kx/kb  float [Ht][Wt], stride cfl_stride: kX and kB of Annex G per
 *              64 x 64 tile (from XFromY / BFromY of C.5.3)
 *   out[c]     [ysize][xsize] of float, uint8 or uint16 (out_format), row
 *              stride out_stride in elements: R, G, B planes. */
typedef struct {
  const int32_t* ac[3];
  size_t ac_stride;
  const int32_t* dc[3];
  size_t dc_stride;
  const uint8_t* strategy;
  const uint8_t* qf_minus_1;
  const uint8_t* sharpness;
  size_t map_stride;
  const float* cfl_kx;
  const float* cfl_kb;
  size_t cfl_stride;
  void* out[3];
  size_t out_stride;
  /* Annex H sums, float [3][2*Hb][2*Wb] (row stride 2*Wb), written by
   * jxlr_ac_prediction and read by jxlr_reconstruct when p->ac_prediction;
   * may be NULL otherwise. */
  const float* ac_pred;
  /* K.5 pseudorandom channels, float [3][ysize][xsize] (row stride xsize),
   * written by jxlr_noise_channels and read by jxlr_finish when p->noise;
   * may be NULL otherwise. */
  const float* noise_raw;
  /* K.3 patches (C.4.6, already decoded): p->num_patches placements of five
   * int32 (x, y, xsize, ysize, offset into patch_samples), each patch's
   * samples int32 [3][ysize][xsize] at its offset; patch_samples_count
   * elements in all.  A placement not inside the frame, larger than 16 or
   * beyond the samples is ill-formed: skipped, with the sticky device flag
   * set (bit 1). */
  const int32_t* patch_place;
  const int32_t* patch_samples;
  size_t patch_samples_count;
  /* K.2 quantized dots (C.4.5, already decoded): p->num_dots of ten int32
   * each: x, y (times 5), sigma_x, sigma_y, angle, sign_intensity,
   * intensity[3], is_circle. */
  const int32_t* dots;
  /* K.4 splines (C.4.7, already decoded, dequantized and recorrelated):
   * spline_offsets int32 [p->num_splines + 1], rising, from 0 to at most
   * p->num_spline_points: spline s has the control points
   * [spline_offsets[s], spline_offsets[s + 1]) of spline_points, int32 (x, y)
   * pairs [p->num_spline_points][2]; spline_dct float [p->num_splines][4][32]:
   * the DCT32 coefficients of X, Y, B and sigma along the arc length.  A
   * spline with no control point, offsets out of range, two consecutive equal
   * control points or an arc length above 2^24 is skipped, with the sticky
   * device flag set (bit 2). */
  const int32_t* spline_offsets;
  const int32_t* spline_points;
  const float* spline_dct;
  /* C.5.2 DcQuantField per channel, float [Hb][Wb], row stride
   * dc_quant_stride elements: the dequantization range of each DC sample
   * (dc_mul[c] / 2^k for the k its decoded delta gives), which the F.2
   * smoothing and the J.3 LLF clamp read.  All three NULL: dc_mul[c] /
   * 2^extra_levels[c] everywhere (the field of a plane whose deltas are all
   * 0; with extra_levels 0 the field whatever the deltas).  Entries must be
   * positive and finite; the library reads them only with dc_smoothing or
   * the quantization constraint on. */
  const float* dc_quant[3];
  size_t dc_quant_stride;
} jxlr_frame_io;

typedef struct jxlr_ctx jxlr_ctx;

/* Human-readable name of a status. */
const char* jxlr_status_string(jxlr_status s);

/* Fills *p with the draft's defaults (C.4.1-C.4.3, C.10, L.2, A.4.5) for a
 * frame of xsize x ysize: global_scale 1, DC weights {4096, 512, 256},
 * x/b_factor_dc = 128, Gaborish on, one EPF pass, F32 output. */
jxlr_status jxlr_params_default(jxlr_frame_params* p, uint32_t xsize, uint32_t ysize);

/* Creates a context on HIP device `device`: builds the dequantization
 * matrices (C.6.1) of the encodings dq[0..14] (a host array indexed by
 * transform type, C.5.4 numbering; NULL: the C.6.1.1 defaults), the
 * transform matrices (I.2.1, I.2.6), LLF tables (I.2.7) and the EPF
 * mul_table (J.2.4) on the host and uploads them.  The encodings are read
 * only during the call.  JXLR_E_DEQUANT: an encoding not valid for its
 * matrix (mode out of range, a 64-entry mode for a larger matrix, band
 * counts out of range, a Copy that does not name an earlier matrix) or a
 * matrix entry that is not positive and finite; JXLR_E_HIP: device
 * allocation or upload failed. */
jxlr_status jxlr_create(jxlr_ctx** ctx, int device, const jxlr_dequant_encoding* dq);
void jxlr_destroy(jxlr_ctx* ctx);

/* Annex G: the chroma-from-luma factors of n u8 XFromY / BFromY values
 * (C.5.3, or x_factor_dc / b_factor_dc of C.4.3): kx[i] = (x_factor[i] -
 * 128) / 256, kb[i] = 0.935669 + (b_factor[i] - 128) / 128.  Host arrays;
 * either pair may be NULL to skip it. */
jxlr_status jxlr_cfl_from_u8(const uint8_t* x_factor, const uint8_t* b_factor, size_t n,
                             float* kx, float* kb);

/* C.4.1: the DC multipliers mX_DC, mY_DC, mB_DC = weight[c] / (global_scale
 * * quant_dc), with weights NULL for the defaults {4096, 512, 256},
 * global_scale = global_scale_minus_1 + 1 (1..65536) and quant_dc =
 * quant_dc_minus_1 + 1 (C.4.2, >= 1).  JXLR_E_PARAM for zero sizes or a
 * weight that is not positive and finite. */
jxlr_status jxlr_dc_mul_from_header(const float* weights, uint32_t global_scale,
                                    uint32_t quant_dc, float dc_mul[3]);

/* Host-side check of host copies of the maps against C.5.4 (every varblock
 * type supported, naturally aligned, inside the frame, no overlap) and C.5.5
 * (quant field uniform within each varblock).  `sharpness` may be NULL;
 * otherwise each entry must be <= 7. */
jxlr_status jxlr_validate_maps_host(const jxlr_frame_params* p, const uint8_t* strategy,
                                    const uint8_t* qf_minus_1, const uint8_t* sharpness,
                                    size_t map_stride);

/* Device workspace jxlr_decode needs for one frame: the block-info map
 * (Hb * Wb bytes) and two sets of XYB float planes (3 * xsize * ysize * 4
 * bytes each; one set when epf_iters == 0), each part 256-byte aligned. */
size_t jxlr_workspace_bytes(const jxlr_frame_params* p);

/* The whole path for one frame: reconstruct, epf_iters EPF passes, Gaborish
 * (if p->gab), XYB -> RGB into io->out.  ws must hold jxlr_workspace_bytes(p). */
jxlr_status jxlr_decode(jxlr_ctx* ctx, const jxlr_frame_params* p, const jxlr_frame_io* io,
                        void* ws, size_t ws_bytes, hipStream_t stream);

/* jxlr_decode for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * workspace is a fixed array in the library's code object, one per device
 * (jxlr_noalloc_scratch_bytes() bytes, 64 MiB: a 1920 x 1080 frame with EPF
 * fits), whose address jxlr_create looks up; the call allocates nothing.
 * Inputs and outputs as for jxlr_decode.  JXLR_E_WORKSPACE (before any
 * launch) when jxlr_workspace_bytes(p) exceeds the array.  Every call on one
 * device shares that device's array: calls that overlap on one device (other
 * streams, other contexts, other host threads) race and give undefined
 * results; calls ordered on one stream are safe. */
jxlr_status jxlr_decode_noalloc(jxlr_ctx* ctx, const jxlr_frame_params* p,
                                const jxlr_frame_io* io, hipStream_t stream);
size_t jxlr_noalloc_scratch_bytes(void);

/* ---- stage entry points (the pieces jxlr_decode runs, for testing and for
 * callers that keep XYB) --------------------------------------------------
 * XYB planes are float [3][ysize][xsize] with row stride xyb_stride elements,
 * plane c at xyb + c * ysize * xyb_stride.  `info` is the block-info map,
 * uint8 [Hb][Wb] (row stride Wb) in device memory owned by the caller. */

/* C.5.4: walks io->strategy (DctSelect) in raster order per 32x32 region and
 * writes, per 8x8 block, its varblock's transform type (bits 0-3) and the
 * block's column and row offset inside the varblock (bits 4-5, 6-7).  Every
 * block of a region with an ill-formed entry (unsupported type, misaligned,
 * out of bounds, overlapping) is written 0xFF and the sticky device flag is
 * set. */
jxlr_status jxlr_block_info(jxlr_ctx* ctx, const jxlr_frame_params* p, const jxlr_frame_io* io,
                            uint8_t* info, hipStream_t stream);

/* Annex H: the predicted sums of every varblock's low coefficients from the
 * DC planes and `info` (F.2 smoothing and DC chroma from luma applied as in
 * the reconstruction) into pred, float [3][2*Hb][2*Wb] in device memory owned
 * by the caller: block (bx, by) holds, at (2 bx + i, 2 by + j), its varblock's
 * coefficient (2 dx + i, 2 dy + j) ((dx, dy): the block's offset inside the
 * varblock; 0 in the LLF corner), scaled like the library's dequantization
 * tables.  Applies whether or not p->ac_prediction is set. */
jxlr_status jxlr_ac_prediction(jxlr_ctx* ctx, const jxlr_frame_params* p, const jxlr_frame_io* io,
                               const uint8_t* info, float* pred, hipStream_t stream);

/* F.2, F.3, Annex G, I.2.7, I.2.4 and the crop of 6.2: coefficient planes of
 * io -> XYB samples, with the varblocks of `info`.  io->out and
 * io->sharpness are not used.  Regions marked ill-formed are written as 0. */
jxlr_status jxlr_reconstruct(jxlr_ctx* ctx, const jxlr_frame_params* p, const jxlr_frame_io* io,
                             const uint8_t* info, float* xyb, size_t xyb_stride,
                             hipStream_t stream);

/* One edge-preserving filter pass (J.2), xyb_in -> xyb_out (distinct buffers).
 * Uses `info`, io->qf_minus_1 and io->sharpness.  Optional debug outputs
 * (NULL to skip): guide bytes uint8 [3][ysize][xsize] (J.2.2) and sigma int32
 * [Hb][Wb] (J.2.4) of this pass.  Pixels of ill-formed regions pass through. */
jxlr_status jxlr_epf_pass(jxlr_ctx* ctx, const jxlr_frame_params* p, const jxlr_frame_io* io,
                          const uint8_t* info, const float* xyb_in, float* xyb_out,
                          size_t xyb_stride, uint8_t* guide_dbg, int32_t* sigma_dbg,
                          hipStream_t stream);

/* Quantization constraint (J.3): xyb_orig holds the input of the first EPF
 * pass, xyb_io the output of the last, which is constrained in place (the two
 * buffers distinct, same stride).  Uses `info` and io->qf_minus_1; applies
 * whether or not p->qco is set.  Pixels of ill-formed regions are left as
 * they are. */
jxlr_status jxlr_qco_pass(jxlr_ctx* ctx, const jxlr_frame_params* p, const jxlr_frame_io* io,
                          const uint8_t* info, const float* xyb_orig, float* xyb_io,
                          size_t xyb_stride, hipStream_t stream);

/* K.3: adds the patches of io to the XYB planes in place (float atomics, so
 * overlapping placements may sum in any order). */
jxlr_status jxlr_patches(jxlr_ctx* ctx, const jxlr_frame_params* p, const jxlr_frame_io* io,
                         float* xyb, size_t xyb_stride, hipStream_t stream);

/* J.4 alone, xyb_in -> xyb_out (distinct buffers): the Gaborish pass that
 * precedes the dots and the splines. */
jxlr_status jxlr_gaborish(jxlr_ctx* ctx, const jxlr_frame_params* p, const float* xyb_in,
                          float* xyb_out, size_t xyb_stride, hipStream_t stream);

/* K.2: dequantizes the dots of io (K.2.1) and adds each over its 5x5 window
 * (samples outside the frame skipped) to the XYB planes in place (float
 * atomics, so overlapping dots may sum in any order).  A set sign bit
 * negates its channel's intensity. */
jxlr_status jxlr_dots(jxlr_ctx* ctx, const jxlr_frame_params* p, const jxlr_frame_io* io,
                      float* xyb, size_t xyb_stride, hipStream_t stream);

/* K.4: renders the splines of io into the XYB planes in place.  Each spline
 * becomes the sequence of points sampling its centripetal Catmull-Rom curve
 * (16 per control point interval, mirrored points extending both ends), the
 * points at unit arc length along the polyline through them (and its last
 * point), and at each such point the ContinuousIDCT of its four coefficient
 * sets at 31 l / L; every pixel whose squared distance from the point is at
 * most -2 sigma^2 log(0.1) gets value d sigma / 4 times the two erf
 * differences over the pixel's extent (a point with sigma <= 0 adds
 * nothing).  Float atomics: overlapping footprints sum in any order.
 * scratch: device memory of at least jxlr_spline_scratch_bytes(p) bytes,
 * owned by the caller, overwritten. */
size_t jxlr_spline_scratch_bytes(const jxlr_frame_params* p);
jxlr_status jxlr_splines(jxlr_ctx* ctx, const jxlr_frame_params* p, const jxlr_frame_io* io,
                         float* xyb, size_t xyb_stride, void* scratch, size_t scratch_bytes,
                         hipStream_t stream);

/* K.5.2: the three pseudorandom channels of every 256x256 group of the frame
 * (frame-sized planes, float [3][ysize][xsize], row stride xsize, device
 * memory owned by the caller); they depend on the frame size only. */
jxlr_status jxlr_noise_channels(jxlr_ctx* ctx, const jxlr_frame_params* p, float* raw,
                                hipStream_t stream);

/* Gaborish (J.4, when p->gab and there are neither dots nor splines), noise (K.5, when
 * p->noise, from io->noise_raw) and XYB -> RGB (L.2) into io->out in
 * p->out_format. */
jxlr_status jxlr_finish(jxlr_ctx* ctx, const jxlr_frame_params* p, const jxlr_frame_io* io,
                        const float* xyb, size_t xyb_stride, hipStream_t stream);

/* The last edge-preserving filter pass (as jxlr_epf_pass from xyb_in)
 * followed by the finish (as jxlr_finish) without storing the pass's
 * output, for a frame with EPF passes and nothing between the last one and
 * the finish: no quantization constraint (J.3) and no patches, dots,
 * splines or noise (Annex K).  Output into io->out in p->out_format, equal
 * bit for bit to jxlr_epf_pass then jxlr_finish.  Each workgroup filters a
 * 64x32 tile, keeps the result on chip and finishes the pixels whose
 * Gaborish window lies in the tile; the samples along tile boundaries go to
 * `seam` (device memory owned by the caller, at least jxlr_seam_bytes(p)
 * bytes, overwritten) and a second launch on the same stream finishes the
 * boundary pixels.  Errors: JXLR_E_PARAM for a frame that does not qualify,
 * JXLR_E_WORKSPACE for a seam buffer below jxlr_seam_bytes(p), and those of
 * jxlr_epf_pass and jxlr_finish.  jxlr_decode takes this path for the last
 * pass of every frame that qualifies. */
jxlr_status jxlr_epf_finish(jxlr_ctx* ctx, const jxlr_frame_params* p, const jxlr_frame_io* io,
                            const uint8_t* info, const float* xyb_in, size_t xyb_stride,
                            float* seam, size_t seam_bytes, hipStream_t stream);

/* The reconstruction (as jxlr_reconstruct) followed by the finish (as
 * jxlr_finish) without an intermediate XYB frame, for a frame whose
 * reconstruction goes to the finish unchanged: no EPF pass (C.10) and no
 * patches, dots, splines or noise (Annex K).  Output into io->out in
 * p->out_format, equal bit for bit to jxlr_reconstruct then jxlr_finish.
 * Each workgroup reconstructs a run of tiles of one tile row into on-chip
 * memory and finishes the pixels whose Gaborish window lies there; the
 * samples along tile-row and run boundaries go to `seam` (device memory
 * owned by the caller, at least jxlr_seam_bytes(p) bytes, overwritten), and
 * a second launch on the same stream finishes the pixels on those
 * boundaries.  Errors: JXLR_E_PARAM for a frame that does not qualify,
 * JXLR_E_WORKSPACE for a seam buffer below jxlr_seam_bytes(p), and those of
 * jxlr_reconstruct and jxlr_finish.  jxlr_decode takes this path for every
 * frame that qualifies. */
jxlr_status jxlr_reconstruct_finish(jxlr_ctx* ctx, const jxlr_frame_params* p,
                                    const jxlr_frame_io* io, const uint8_t* info, float* seam,
                                    size_t seam_bytes, hipStream_t stream);

/* Bytes of the seam buffer that jxlr_epf_finish and jxlr_reconstruct_finish
 * take for frame p: the samples of each 64x32 tile's outer two rows and
 * columns in all three channels (4.5 KiB per tile), rounded up to 256 bytes;
 * 0 for a frame that qualifies for neither fused path. */
size_t jxlr_seam_bytes(const jxlr_frame_params* p);

/* ---- JPEG1 direct rasterization (M.6) ----------------------------------------
 * A recompressed JPEG1 frame (M.4 already decoded: quantized DCT coefficients
 * per component and the quantization tables) straight to RGB: dequantization
 * (M.6.1) and IDCT (M.6.2) per component, the gated Gaborish of the M.6.3
 * side channel when present, 2x linear upsampling of subsampled components
 * (M.6.4), YCbCr -> RGB (M.6.5) and the crop (M.6.6).  Not done: the other
 * optional side channels (coefficient conditioning M.6.1.1, HDR colour
 * spaces M.6.5.1).  Errors, all synchronous and
 * before any launch: JXLR_E_NULL for a missing pointer; JXLR_E_PARAM for a
 * component count other than 1 or 3, a sampling factor outside {1, 2} or
 * above component 0's, a quantization step outside 1..65535 or a component
 * index out of range; JXLR_E_SIZE for sizes outside 1..65536 or strides
 * below a plane's width (and, for pix, not a multiple of 4 or not 16-byte
 * aligned); JXLR_E_WORKSPACE for a workspace below
 * jxlr_jpeg1_workspace_bytes.  All buffers are the caller's device memory. */
typedef struct {
  int32_t xsize, ysize;       /* image size in pixels, 1..65536 */
  int32_t num_components;     /* 1 (grey) or 3 (Y, Cb, Cr) */
  int32_t h_samp[3], v_samp[3]; /* sampling factors 1 or 2; component 0 the largest */
  int32_t quant[3][64];       /* quantization steps 1..65535, index 8 u + v */
  /* M.6.3 side channel ("BRN:GAB"): 1 if present, applied after the IDCT of
   * every component; gab_code[c] holds the component's four decoded bytes:
   * gab_weight1 * 1024, gab_weight2 * 1024, threshold * 16, limit. */
  int32_t gab;
  uint8_t gab_code[3][4];
} jxlr_jpeg1_params;

/* Blocks of component c: whole MCUs of 8 h_samp[0] x 8 v_samp[0] pixels
 * cover the image, and component c has h_samp[c] x v_samp[c] blocks per MCU. */
jxlr_status jxlr_jpeg1_blocks(const jxlr_jpeg1_params* p, int32_t c, int32_t* wib, int32_t* hib);

/* Device workspace of jxlr_jpeg1_decode: one float plane per component, two
 * with the M.6.3 side channel (0 if p is invalid). */
size_t jxlr_jpeg1_workspace_bytes(const jxlr_jpeg1_params* p);

/* M.6.3 for component c with its side-channel bytes p->gab_code[c]
 * (whatever p->gab says): the J.4 smoothing of pix_in (3x3 kernel, centre 1,
 * edge gab_weight1, diagonal gab_weight2, normalized; mirrored at the
 * plane's edges), then per 8x8 block the smoothed values when fewer than
 * limit of the block's 6x6 interior pixels (offsets 1..6) differ from them
 * by more than the threshold, else the block's own, into pix_out.  Planes
 * as jxlr_jpeg1_idct writes them (float [8 hib][8 wib], strides multiples
 * of 4, pointers 16-byte aligned), distinct (JXLR_E_PARAM otherwise). */
jxlr_status jxlr_jpeg1_gaborish(jxlr_ctx* ctx, const jxlr_jpeg1_params* p, int32_t c,
                                const float* pix_in, size_t in_stride, float* pix_out,
                                size_t out_stride, hipStream_t stream);

/* M.6.1-M.6.2 for component c: coef int32 [8 hib][8 wib] device memory, row
 * stride coef_stride elements, coefficient 8 u + v of block (bx, by) at row
 * 8 by + u, column 8 bx + v (u the vertical frequency; JPEG1's natural
 * order); each is multiplied by quant[c][8 u + v] and I(8, u) I(8, v)
 * (I.2.6.1) and the block goes through IDCT_2D (I.2.2).  pix: float
 * [8 hib][8 wib], row stride pix_stride elements (a multiple of 4, the
 * pointer 16-byte aligned), level shift not applied. */
jxlr_status jxlr_jpeg1_idct(jxlr_ctx* ctx, const jxlr_jpeg1_params* p, int32_t c,
                            const int32_t* coef, size_t coef_stride, float* pix, size_t pix_stride,
                            hipStream_t stream);

/* M.6.4-M.6.6: components of pix[c] (planes of jxlr_jpeg1_idct) upsampled
 * 2x where their factor is half component 0's (horizontally first; 3/4 of
 * the nearest sample and 1/4 of the next one out, mirrored at the plane's
 * edges), then R = 1.402 Cr + (Y + 128), G = -0.71414 Cr - 0.34414 Cb +
 * (Y + 128), B = 1.772 Cb + (Y + 128) (grey: all three Y + 128), cropped to
 * xsize x ysize: rgb[3] float [ysize][xsize] with row stride rgb_stride. */
jxlr_status jxlr_jpeg1_color(jxlr_ctx* ctx, const jxlr_jpeg1_params* p, const float* const pix[3],
                             const size_t pix_stride[3], float* const rgb[3], size_t rgb_stride,
                             hipStream_t stream);

/* The whole rasterization: jxlr_jpeg1_idct of every component into ws, with
 * p->gab jxlr_jpeg1_gaborish of each into the second half of ws, then
 * jxlr_jpeg1_color.  coef / coef_stride as for jxlr_jpeg1_idct, per
 * component (entries past num_components ignored). */
jxlr_status jxlr_jpeg1_decode(jxlr_ctx* ctx, const jxlr_jpeg1_params* p,
                              const int32_t* const coef[3], const size_t coef_stride[3],
                              float* const rgb[3], size_t rgb_stride, void* ws, size_t ws_bytes,
                              hipStream_t stream);

/* ---- batches of frames ------------------------------------------------------
 * A batch decodes n independent frames (each with its own sizes, parameters,
 * options and inputs) in one launch per stage: the tiles of all frames form
 * one list that persistent workgroups walk, so small frames share the GPU
 * instead of each leaving most of it idle.  The options (AC prediction, the
 * quantization constraint, patches, noise, dots, splines) run as option
 * stages: one launch each over the frames that use it.  Results are
 * bit-identical to jxlr_decode of each frame alone. */

/* Stages of a batch, for jxlr_batch_stage, in the order jxlr_batch_run
 * runs them: INFO (every frame); PRED (Annex H); FUSED (the frames
 * jxlr_reconstruct_finish qualifies: reconstruction to output); the tile
 * stages RECON and EPF (every other frame; a frame with fewer passes sits
 * out the later ones, and the last pass of a frame jxlr_epf_finish
 * qualifies also finishes it); SEAM (the boundary pixels of both fused
 * kinds); QCO (J.3), PATCHES (K.3), NOISE (K.5 channels), GABORISH (J.4 as
 * its own pass, for frames with dots or splines), DOTS (K.2), SPLINES (K.4);
 * FINISH (the frames not finished by then).  Each option stage takes the
 * frames that use it. */
enum {
  JXLR_STAGE_INFO = 0, JXLR_STAGE_RECON = 1, JXLR_STAGE_EPF = 2, JXLR_STAGE_FINISH = 3,
  JXLR_STAGE_PRED = 4, JXLR_STAGE_QCO = 5, JXLR_STAGE_PATCHES = 6, JXLR_STAGE_NOISE = 7,
  JXLR_STAGE_GABORISH = 8, JXLR_STAGE_DOTS = 9, JXLR_STAGE_SPLINES = 10,
  JXLR_STAGE_FUSED = 11, JXLR_STAGE_SEAM = 12
};
#define JXLR_BATCH_OPT_STAGES 9 /* JXLR_STAGE_PRED .. JXLR_STAGE_SEAM */

/* Device workspace for a batch: a descriptor header plus, per frame, what
 * jxlr_workspace_bytes(&p[i]) names; 0 if n <= 0 or a parameter set is out of
 * range. */
size_t jxlr_batch_workspace_bytes(int n, const jxlr_frame_params* p);

/* Filled by jxlr_batch_prepare; describes a batch written into `ws`. */
typedef struct jxlr_batch_plan {
  void* ws;
  size_t ws_bytes;
  int n;
  int total_tiles;   /* 64x32 pixel tiles over the frames outside FUSED */
  int total_regions; /* 32x32 DctSelect regions over all frames */
  int max_epf_iters;
  size_t frames_offset, tile_frame_offset, tile_start_offset, region_start_offset;
  int any_split;     /* some frame has idct_split set */
  int any_noise;     /* some frame adds noise */
  /* option stage JXLR_STAGE_PRED + k: the frames that take it, its
   * workgroups over them, and where its table and unit prefix sit in ws */
  int opt_frames[JXLR_BATCH_OPT_STAGES];
  int opt_units[JXLR_BATCH_OPT_STAGES];
  size_t opt_entries_offset[JXLR_BATCH_OPT_STAGES];
  size_t opt_start_offset[JXLR_BATCH_OPT_STAGES];
} jxlr_batch_plan;

/* Schedule of the four persistent stage kernels.  grid_*: workgroup count;
 * 0 picks one workgroup per tile (per 256 regions for the block-info stage)
 * and larger values are clamped down to that.  order_*: 0 strided (tile t to
 * workgroup t mod grid); 1 XCD-contiguous (each of the eight XCDs takes about
 * one contiguous eighth of the tile list, so neighbouring tiles share an L2).
 * The output does not depend on the schedule. */
typedef struct jxlr_launch_config {
  int grid_info;
  int grid_recon;
  int grid_epf;
  int grid_finish;
  int order_recon;
  int order_epf;
  int order_finish;
} jxlr_launch_config;

/* Validates every frame as the single-frame entry points do and writes the
 * batch descriptors into `ws` (device memory, ws_bytes >=
 * jxlr_batch_workspace_bytes(n, p)).  The copies are ordered on `stream`
 * (after any earlier work on it, such as a previous batch still reading the
 * same workspace) and the call waits for them, so it synchronizes `stream`;
 * a workspace reused on another stream must be free of that stream's work
 * first.  p[i] and io[i] are host arrays of n entries; the device buffers
 * io[i] names must stay valid while the plan is run.  Calls no kernel. */
jxlr_status jxlr_batch_prepare(jxlr_ctx* ctx, int n, const jxlr_frame_params* p,
                               const jxlr_frame_io* io, void* ws, size_t ws_bytes,
                               jxlr_batch_plan* plan, hipStream_t stream);

/* Enqueues the whole path for every frame of the plan on `stream`: block
 * info, AC prediction, the fused reconstruction and finish with its seam
 * pass, reconstruction, max_epf_iters EPF passes (a frame with fewer passes
 * sits out the rest), the option stages from QCO to SPLINES, and finish; a
 * stage that no frame takes launches nothing.  cfg may be NULL. */
jxlr_status jxlr_batch_run(jxlr_ctx* ctx, const jxlr_batch_plan* plan,
                           const jxlr_launch_config* cfg, hipStream_t stream);

/* Enqueues one stage of a prepared batch (EPF: pass epf_pass, reading and
 * writing the XYB buffers that pass uses; option stages ignore grid and
 * order).  Each stage reads what the stage before it wrote, so stages must
 * run in jxlr_batch_run's order for a correct result.  Repeating one tile
 * stage alone is idempotent; QCO, PATCHES, DOTS and SPLINES change their
 * buffer in place and are not. */
jxlr_status jxlr_batch_stage(jxlr_ctx* ctx, const jxlr_batch_plan* plan, int stage, int grid,
                             int order, int epf_pass, hipStream_t stream);

/* Autotuner: picks, per tile stage, the workgroup count and tile order with
 * the shortest time on this device for this batch.  Candidates: one
 * workgroup per tile, and persistent grids of 1-4 times (compute units x
 * resident workgroups per compute unit) in both orders; each timed with HIP
 * events as the best of three groups of `reps` launches.  Runs the batch
 * before and after (its outputs are written as by jxlr_batch_run) and
 * synchronizes `stream`.  best_ms (may be NULL) receives the tuned stage time
 * sum of one run, EPF counted max_epf_iters times. */
jxlr_status jxlr_autotune(jxlr_ctx* ctx, const jxlr_batch_plan* plan, int reps,
                          jxlr_launch_config* best, float* best_ms, hipStream_t stream);

/* jxlr_batch_prepare (on `stream`) followed by jxlr_batch_run with the
 * default config. */
jxlr_status jxlr_decode_batch(jxlr_ctx* ctx, int n, const jxlr_frame_params* p,
                              const jxlr_frame_io* io, void* ws, size_t ws_bytes,
                              hipStream_t stream);

/* A prepared batch captured once into a HIP graph, for callers that replay the
 * same batch shape (the plan's buffers are fixed; refill their contents
 * between launches).  The capture uses a private default-priority stream and
 * records kernel nodes only. */
typedef struct jxlr_graph jxlr_graph;
jxlr_status jxlr_graph_create(jxlr_ctx* ctx, const jxlr_batch_plan* plan,
                              const jxlr_launch_config* cfg, jxlr_graph** out);
jxlr_status jxlr_graph_launch(jxlr_graph* g, hipStream_t stream);
void jxlr_graph_destroy(jxlr_graph* g);

/* Reads and clears (in one atomic exchange on the device, ordered on
 * `stream`) the sticky device-validation flag: JXLR_OK or
 * JXLR_E_DEVICE_VALIDATION.  Synchronizes `stream`.  The flag belongs to the
 * context: every call on the context sets the same flag, whatever its
 * stream, so with calls in flight on several streams a set flag does not
 * say which call set it.  Callers that need the flag per request use a
 * context per stream, or check the maps on the host first
 * (jxlr_validate_maps_host). */
jxlr_status jxlr_get_device_status(jxlr_ctx* ctx, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif
