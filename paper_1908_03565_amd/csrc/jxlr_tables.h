// Host-built constant tables of the VarDCT reconstruction library, and the
// device-side layout they are uploaded in.
#pragma once

#include <cstdint>

namespace jxlr {

// Number of transform types the library reconstructs (C.5.4 values 0..14).
constexpr int kNumStrategies = 15;

// Varblock size in 8x8 blocks of transform type s (I.2.5: "DCT N x M" is
// max(8, N) wide and max(8, M) tall).
inline int blocks_x(int s) {
  static const int8_t w[15] = {1, 1, 1, 1, 2, 4, 2, 1, 4, 1, 4, 2, 1, 1, 1};
  return w[s];
}
inline int blocks_y(int s) {
  static const int8_t h[15] = {1, 1, 1, 1, 2, 4, 1, 2, 1, 4, 2, 4, 1, 1, 1};
  return h[s];
}

// Offsets (in floats) of the per-type dequantization matrices inside
// DeviceTables::dq; channel c of type s starts at dq_offset(s) + c * bx * by.
int dq_offset(int s);
// Buckets of binary32 values for the 8-bit output code: bucket b holds the
// values whose bit pattern shifted right by 16 (sign, exponent and the top 7
// mantissa bits) is kSrgbBucket0 + b, from 2^-14 up to 1.0 (b = 0 also takes
// every smaller value).
constexpr int kSrgbBucket0 = (127 - 14) << 7;
constexpr int kSrgbBuckets = (127 << 7) - kSrgbBucket0 + 1;
constexpr int kSrgbBucketsPadded = (kSrgbBuckets + 3) & ~3;
constexpr int kDqFloats = 3 * (4 * 64 + 256 + 1024 + 2 * 128 + 2 * 256 + 2 * 512 + 3 * 64);

// Everything the kernels read that does not depend on the frame.  One
// instance lives in device memory per context.
struct DeviceTables {
  // Inverse 1-D transform matrices, row n = output sample, column k = input
  // coefficient (I.2.1 and the generated transforms).
  float t8[8 * 8];
  float t16[16 * 16];
  float t32[32 * 32];
  // DCT4x4 separable pass on an 8-vector (I.2.4.3): two interleaved 4-point
  // inverse transforms; m4[4 s + j][s + 2 i] = T4[j][i].
  float m4[8 * 8];
  // LLF from DC (I.2.7.2), one axis: a16[x][i] for 2 DC samples of a
  // 16-pixel side, a32[x][i] for 4 samples of a 32-pixel side, with the
  // ScaleF factor and the 1 / (samples) division folded in.
  float a16[2 * 2];
  float a32[4 * 4];
  // Dequantization matrices (C.6.1, defaults of C.6.1.1), row-major [y][x].
  float dq[kDqFloats];
  // The same matrices multiplied by the per-frequency scales of the inverse
  // transforms (s_N(y) s_N(x); for DCT4 the 4-point scales of the
  // interleaved sub-blocks; 1 for DCT2 and Identity), so that the kernels
  // run the plain DCT-III y_n = sum_k x_k cos(pi (2n + 1) k / (2N)).
  float dqs[kDqFloats];
  // a16 / a32 with the same scale applied to the output frequency x.
  float a16s[2 * 2];
  float a32s[4 * 4];
  // mul_table of J.2.4 for sigma 0..672 (entries below 16 unused), one per
  // kSigmaShift value 0..8.
  int32_t mul_table[9][673];
  // Decision thresholds of the 8- and 16-bit outputs (sRGB transfer function
  // of clamp(v, 0, 1), then floor(e (2^b - 1) + 0.5), evaluated in binary64):
  // srgb_thrB[k], k = 1 .. 2^B - 1, is the smallest binary32 v whose code is
  // at least k; entry 0 is -inf and entry 2^B is +inf.  The code of v is the
  // c with srgb_thrB[c] <= v < srgb_thrB[c + 1].
  float srgb_thr8[257];
  float srgb_thr16[65537];
  // 8-bit code of the smallest value of each bucket (see kSrgbBucket0); no
  // bucket spans more than two codes (checked when the table is built), so
  // the code of v is start + (v >= srgb_thr8[start + 1]).
  alignas(4) uint8_t srgb_start8[kSrgbBucketsPadded];
  // Split-precision transform operands: the plain DCT-III matrix of a
  // 32-sample region side made of 32 / N diagonal N-point blocks (m = 0, 1, 2
  // for N = 8, 16, 32), A[i][k] = cos(pi (2 (i mod N) + 1)(k mod N) / (2 N))
  // when i / N == k / N, else 0, times 16 (so that the rests of the smallest
  // cosines stay normal numbers), as binary16 bit patterns of its high part
  // (part 0, rounded to nearest even) and of the rest (part 1), in the
  // A-operand order of a 32x32x16 matrix instruction: element e of lane l in
  // k-step t is A[l mod 32][16 t + 8 (l / 32) + e].  The split form's A
  // operands.
  alignas(16) uint16_t mfma_h[3][2][2][64][8];
  // The same cosines in binary32 for the varblocks' LLF corners, which the
  // split form transforms outside the matrix products: llf_cos[m][n][u] =
  // cos(pi (2 n + 1) u / (2 N)), N = 8 << m, n < N, u < 4 (zero for u >= N / 8),
  // and llf_c1[m][n] = llf_cos[m][n][1].
  alignas(16) float llf_cos[3][32][4];
  float llf_c1[3][32];
  // AFV basis (I.2.2): afv[j][i] = basis vector j at 4x4 index i.
  float afv[16][16];
  // Inverses of a16s and a32s: DC samples from the scaled LLF, one axis
  // (quantization constraint, J.3).
  float b16s[2 * 2];
  float b32s[4 * 4];
  // AC prediction (Annex H), one axis of a varblock side of 8 n pixels
  // (m = 0, 1, 2 for n = 1, 2, 4 DC samples): pred_u[m][j][i], the mean of
  // 4-pixel cell j of the side decoded from its LLF, from DC sample i
  // (I.2.7 then I.2.6 at N = 4); pred_v[m][k][j], coefficient k < 2n from
  // the 2n cells (I.2.7 at N = 4, the inverse of the cell means of the
  // lowest 2n frequencies), times the scale s_N(k) of the passes.
  float pred_u[3][8][4];
  float pred_v[3][8][8];
  // ScaleF(2, 8, 1) of the DCT4x8 / DCT8x4 forms of I.2.7.3, and the pass
  // scale s_8(1) of their 8-point axis.
  float pred_sf;
  float pred_s8_1;
  // Noise (K.5.2): jump-ahead of one XorShift128+ generator, whose 128-bit
  // state (bits 0-63 the first word, 64-127 the second) advances by a map
  // linear over GF(2).  noise_nib[k][p][v] is the image under that map's
  // 2^k-th power of the state whose nibble p (bits 4p .. 4p + 3) is v and
  // whose other bits are 0, as two words; the image of a state is the XOR
  // of the entries its 32 nibbles select.
  uint64_t noise_nib[14][32][16][2];
  // Splines (K.4): DCTScale(k) of ContinuousIDCT, D(32, k) of I.2.6.1 times
  // 1 / (4 sqrt 2) at k = 0 and 1/4 elsewhere, in binary64.
  double spline_scale[32];
  // JPEG1 rasterization (M.6.1-M.6.2): jpeg1_a[y][u] is IDCT_1D's entry
  // (I.2.1) times I(8, u) (I.2.6.1), rounded once from binary64.
  float jpeg1_a[8][8];
};

// Encoding of one dequantization matrix (C.6.1): the layout of the public
// jxlr_dequant_encoding (checked where both are visible).
enum DequantMode {
  kDqLibrary = 0, kDqIdentity = 1, kDqDct2 = 2, kDqDct4 = 3, kDqDct4x8 = 4, kDqAfv = 5,
  kDqDct = 6, kDqCopy = 7
};
struct DequantEncoding {
  int32_t mode;
  int32_t copy_from;
  int32_t num_bands;
  int32_t num_ecc_bands;
  double dist_bands[3][17];
  double ecc_bands[3][8];
  double params[3][6];
  double afv_weights[3][8];
};

// Fills t on the host, with the dequantization matrices of the encodings
// enc[0..14] (indexed by transform type; null: the C.6.1.1 defaults).
// Returns false if an encoding is not valid for its matrix or an entry is
// not positive and finite (C.6.1).
bool build_tables(DeviceTables* t, const DequantEncoding* enc = nullptr);

// The C.6.1.1 default encoding of transform type s.
void default_encoding(int s, DequantEncoding* out);
// The same tables in double precision, for the host-side cross-checks.
bool dequant_matrix_f64(int s, int c, double* out, const DequantEncoding* enc = nullptr);
void inverse_transform_matrix_f64(int n, double* out);
// s_N(k): the draft's inverse transform is the plain DCT-III applied to
// coefficients multiplied by s_N(k).
double transform_scale(int n, int k);
void epf_mul_table(int sigma_shift, int32_t* table);
// The output code of a binary32 sample, in binary64 (bits = 8 or 16).
int srgb_code_f64(int bits, float v);
// Fills thr[0 .. 2^bits] as described for DeviceTables::srgb_thr8/16.
void srgb_thresholds(int bits, float* thr);
// Fills DeviceTables::srgb_start8; false if a bucket spans more than two codes.
bool srgb_bucket_starts(uint8_t* start);
// binary16 bit pattern of v rounded to nearest, ties to even (finite v
// within the binary16 range), and its value.
uint16_t f16_rne(double v);
double f16_value(uint16_t h);

}  // namespace jxlr
