// Test-only shim: exposes the library's host-built constant tables to the
// CPU tests, which compare them with the oracle's independently built ones.
#include <cstddef>
#include <cstdint>

#include "jxlr_tables.h"

static jxlr::DeviceTables g_tables;

extern "C" {
int shim_dequant(int s, int c, double* out) { return jxlr::dequant_matrix_f64(s, c, out) ? 1 : 0; }
void shim_inverse(int n, double* out) { jxlr::inverse_transform_matrix_f64(n, out); }
void shim_mul_table(int shift, int32_t* t) { jxlr::epf_mul_table(shift, t); }
int shim_build() { return jxlr::build_tables(&g_tables) ? 1 : 0; }
int shim_dequant_enc(int s, int c, const void* enc, double* out) {
  return jxlr::dequant_matrix_f64(s, c, out, static_cast<const jxlr::DequantEncoding*>(enc)) ? 1 : 0;
}
int shim_encoding_size() { return int(sizeof(jxlr::DequantEncoding)); }
const float* shim_t8() { return g_tables.t8; }
const float* shim_t16() { return g_tables.t16; }
const float* shim_t32() { return g_tables.t32; }
const float* shim_m4() { return g_tables.m4; }
const float* shim_a16() { return g_tables.a16; }
const float* shim_a32() { return g_tables.a32; }
const float* shim_dq() { return g_tables.dq; }
const float* shim_dqs() { return g_tables.dqs; }
const float* shim_a16s() { return g_tables.a16s; }
const float* shim_a32s() { return g_tables.a32s; }
const int32_t* shim_mul(int shift) { return g_tables.mul_table[shift]; }
int shim_dq_offset(int s) { return jxlr::dq_offset(s); }
const uint16_t* shim_mfma(int m) { return &g_tables.mfma_h[m][0][0][0][0]; }
const float* shim_thr(int bits) { return bits == 8 ? g_tables.srgb_thr8 : g_tables.srgb_thr16; }
const uint8_t* shim_start8() { return g_tables.srgb_start8; }
int shim_bucket0() { return jxlr::kSrgbBucket0; }
int shim_buckets() { return jxlr::kSrgbBuckets; }
const float* shim_afv() { return &g_tables.afv[0][0]; }
const float* shim_b16s() { return g_tables.b16s; }
const float* shim_b32s() { return g_tables.b32s; }
const float* shim_pred_u() { return &g_tables.pred_u[0][0][0]; }
const float* shim_pred_v() { return &g_tables.pred_v[0][0][0]; }
float shim_pred_sf() { return g_tables.pred_sf; }
float shim_pred_s8_1() { return g_tables.pred_s8_1; }
const uint64_t* shim_noise_nib() { return &g_tables.noise_nib[0][0][0][0]; }
const double* shim_spline_scale() { return g_tables.spline_scale; }
}
