// Constant tables of the VarDCT reconstruction library, built on the host in
// double precision and stored as binary32 for the kernels.
//
//   - inverse transform matrices (I.2.1 and the generated transforms), derived
//     from the scale factors of I.2.6.1: T_N = Q_N diag(1 / I(N, k)) where Q_N
//     is the orthonormal DCT-III;
//   - LLF-from-DC factors (I.2.7.2);
//   - default dequantization matrices (C.6.1, C.6.1.1);
//   - the EPF mul_table (J.2.4).
#include "jxlr_tables.h"

#include <algorithm>
#include <cmath>
#include <limits>
#include <cstring>
#include <vector>

namespace jxlr {
namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;

// I.2.6.1 building blocks.
double i8(int n, int u) {
  const double eps = u == 0 ? std::sqrt(0.5) : 1.0;
  return std::sqrt(2.0 / n) * eps * std::cos(u * kPi / (2.0 * n));
}
double d8(int n, int u) { return 1.0 / (n * i8(n, u)); }
double scale_i(int n, int u) { return n == 8 ? i8(n, u) : d8(n, u); }
double scale_d(int n, int u) { return n == 8 ? d8(n, u) : i8(n, u); }
// C(N, n, x): product of cos(x pi / (2 m)) for m = N, N/2, ... above n, or
// its reciprocal when n > N.
double scale_c(int N, int n, int x) {
  if (n > N) return 1.0 / scale_c(n, N, x);
  double v = 1.0;
  for (int m = N; m > n; m /= 2) v *= std::cos(x * kPi / (2.0 * m));
  return v;
}
// ScaleF(N, n, x) of I.2.6.1.
double scale_f(int N, int n, int x) {
  return std::sqrt(double(N) * n) * scale_d(N, x) * scale_i(n, x) * scale_c(N, n, x);
}

// Orthonormal DCT-III: q[n][k].
double ortho(int n_size, int n, int k) {
  const double a = std::sqrt((k == 0 ? 1.0 : 2.0) / n_size);
  return a * std::cos(kPi * (2 * n + 1) * k / (2.0 * n_size));
}

// ------------------------------------------------------------------------
// Dequantization encodings of C.6.1.1 (channel X, Y, B).
struct BandSet {
  int n;
  double v[3][8];
};

const BandSet kDist8 = {6, {{5.0, 0.0, -0.4, -0.4, -0.4, -2.0},
                            {1.1, 0.0, -0.3, -0.3, -0.3, -0.3},
                            {1.0, -3.0, 0.0, 0.0, -1.0, -2.0}}};
const BandSet kDist4 = {4, {{32.0, -0.4, 0.0, 0.0}, {6.0, 0.0, 0.0, -0.0}, {4.0, -5.0, -1.0, -1.0}}};
const double kDct4Mul[3][2] = {{1.0, 1.0}, {0.7, 0.7}, {1.0, 1.0}};
const BandSet kDist16 = {7,
                         {{3.1965020925735868, -1.8000777393353804, -0.39424529824571225,
                           -0.33909377445710343, -0.6350101832695744, -0.90177264050827612,
                           -1.5162099239887414},
                          {0.77917081615440487, -0.57424582104194355, -0.90745813428471001,
                           -0.64925837484843441, -0.35865440981033403, -0.21322389111877305,
                           -0.27615025315725483},
                          {0.22259376988644336, -3.0531423165804414, -0.2, -0.30687130033378396,
                           -0.42708730624733904, -1.4856834539296244, -5.9209142884401604}}};
const BandSet kDist32 = {8,
                         {{0.47968775359573942, -1.025, -0.98, -0.9012, -0.4, -0.48819395464,
                           -0.421064, -0.27},
                          {0.22295421389982905, -0.8041958212306401, -0.7633036457487539,
                           -0.55660379990111464, -0.49785304658857626, -0.43699592683512467,
                           -0.40180866526242109, -0.27321683125358037},
                          {0.11607457694128877, -3.060733579805728, -2.0413270132490346,
                           -2.0235650159727417, -0.5495389509954993, -0.4, -0.4, -0.3}}};
const BandSet kDist16x8 = {7, {{5.0, -0.7, -0.7, -0.2, -0.2, -0.2, -0.5},
                               {1.0, -0.5, -0.5, -0.5, -0.2, -0.2, -0.2},
                               {0.35, -1.4, -0.2, -0.5, -0.5, -1.5, -3.6}}};
const BandSet kDist32x8 = {8,
                           {{0.90897201669289496, -2.523575079652864, 1.5606102630460328,
                             -0.6828050717528521, -14.770016895841904, -31.365240527393656,
                             0.565929254166433, 26.789646874558219},
                            {0.3603042187746216, -0.11724474917749789, -0.85426302204085935,
                             -0.5404181207241352, -0.45637619443533173, -0.82707923060149569,
                             -1.09760551067614, -54.16057009483842},
                            {0.25176400522276937, -10.060949304689093, -4.5316627381323995,
                             -5.4569229849460807, -10.549754675878864, 1.7512906265092971,
                             -1.6854706115725824, 3.3092762331901451}}};
const BandSet kEcc32x8 = {4,
                          {{-0.40751133465833289, 2.2055690721475925, -1.4434547377534228,
                            2.0590289434445102},
                           {0.12452072219659419, 0.065578935001406033, -0.14598888885596958,
                            0.12114139909222557},
                           {0.0586589025020419, -2.2654958780302183, -4.6996221931893647,
                            1.8254498073137184}}};
const BandSet kDist32x16 = {8,
                            {{1.1280371559733287, -0.98868, -0.658, -0.42026, -0.22712, -0.2206,
                              -0.226, -0.2},
                             {0.38961075971152237, -0.62525308982767058, -0.83770786552491361,
                              -0.79014862079498627, -0.2692727459704829, -0.38272769465388551,
                              -0.2292422253091453, -0.20719098826199578},
                             {0.098, -2.41, -0.23, -0.2, -0.4, -0.8, -0.4, -0.5}}};
// DCT4x8 mode (DCT4x8, and transposed DCT8x4): four distance bands, two
// eccentricity bands of zero, one multiplier per channel.
const BandSet kDist4x8 = {4,
                          {{17.142628543359718, -0.16269623020744692, -0.31194253026666783,
                            -0.2151140670773547},
                           {4.6225628588812384, -0.82630200888366945, -1.0675229603596517,
                            -0.17845290869168118},
                           {0.81188546639482984, -0.6594385811273854, -0.050082094097871593,
                            -2.6843722511996204}}};
const double kDct4x8Mul[3] = {1.0, 1.0, 1.0};
// AFV mode: afv_weights (four 2x2-group weights, the first band value and
// three band parameters) and the two multipliers, per channel; the
// frequency of each 4x4 position and the range they are mapped from.
const double kAfvW[3][8] = {
    {6368.834817724610816928, 232.1096058872860158351, 415.663547479750900044,
     220.0720486370546864556, 329.818962738766012564, -0.9919974139384578, 0, -0.60},
    {1608.323575150649711025, 67.2724358236086, 89.06657498438612, 64.07248898359674,
     125.6541247697168638611, -2.2833978673775697, -0.14, -0.2485},
    {195.927828574730424638, 21.841306388764952, 18.5279466567289584105, 12.573868715940659,
     15.89916083965558, -0.41, -0.1608, 0}};
const double kAfvMul[3][2] = {{1.0, 1.0}, {1.0, 1.0}, {1.0, 1.0}};
const double kAfvFreq[16] = {0, 0, 0.8517778890324296, 5.37778436506804, 0, 0,
                             4.734747904497923, 5.449245381693219, 1.6598270267479331, 4,
                             7.275749096817861, 10.423227632456525, 2.662932286148962,
                             7.630657783650829, 8.962388608184032, 12.97166202570235};
const double kAfvLo = 0.8517778890324296, kAfvHi = 12.1198851366699204;
// The AFV basis (I.2.2), vector i = row i, 4x4 entry (x, y) at 4 y + x; the
// two rows printed with 17 entries are taken with their spurious zero
// removed (row 4 the last, row 9 the one at index 3), which makes the basis
// orthonormal.
const double kAfvBasis[16][16] = {
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
const double kIdentityW[3][3] = {{221.50801256717435, 7087.151589594002, 4466.9924939259863},
                                 {29.535505378287006, 1454.6663024982124, 1368.041230099175},
                                 {9.2887405354132238, 23.982311358829531, 11.201853748207084}};
const double kDct2W[3][6] = {{3840.0, 2560.0, 1280.0, 640.0, 480.0, 300.0},
                             {960.0, 640.0, 320.0, 180.0, 140.0, 120.0},
                             {640.0, 320.0, 128.0, 64.0, 32.0, 16.0}};

// Band multiplier of an encoded band value (C.6.1).
double band_mult(double v) { return v > 0 ? 1.0 + v : 1.0 / (1.0 - v); }

// Cumulative band values: element 0 is `first`, each later one multiplies in
// the next encoded value.
std::vector<double> cumulative(double first, const double* enc, int count) {
  std::vector<double> out(1, first);
  for (int i = 0; i < count; ++i) out.push_back(out.back() * band_mult(enc[i]));
  return out;
}

// Geometric interpolation between band points; positions at or beyond the
// last point take the last value.
double interp(double pos, double span, const std::vector<double>& pts) {
  const int last = int(pts.size()) - 1;
  const double sp = pos * last / span;
  const double fl = std::floor(sp);
  if (fl >= last) return pts[last];
  const int i = int(fl);
  return pts[i] * std::pow(pts[i + 1] / pts[i], sp - fl);
}

// DCT-mode weight matrix for X columns and Y rows, row-major, from nb
// encoded distance bands and ne encoded eccentricity bands.
std::vector<double> band_weights(int X, int Y, const double* db, int nb, const double* eb,
                                 int ne) {
  // distance bands: db[0], then one multiplier per further encoded value
  std::vector<double> dpts = cumulative(db[0], db + 1, nb - 1);
  std::vector<double> epts = cumulative(1.0, eb, ne);
  std::vector<double> w(size_t(X) * Y);
  for (int y = 0; y < Y; ++y) {
    for (int x = 0; x < X; ++x) {
      const double u = double(x) / X, v = double(y) / Y;
      const double dist_v = std::hypot(u, v);
      double m = interp(dist_v, std::sqrt(2.0), dpts);
      if (x || y) m *= interp(std::fabs(u - v) / dist_v, 1.0, epts);
      w[size_t(y) * X + x] = m;
    }
  }
  return w;
}

void set_bands(DequantEncoding* e, const BandSet& dist, const BandSet* ecc, int n_ecc) {
  e->num_bands = dist.n;
  e->num_ecc_bands = n_ecc;
  for (int c = 0; c < 3; ++c) {
    for (int i = 0; i < dist.n; ++i) e->dist_bands[c][i] = dist.v[c][i];
    for (int i = 0; i < n_ecc; ++i) e->ecc_bands[c][i] = ecc ? ecc->v[c][i] : 0.0;
  }
}

// The encoding matrix s is built from: Library is the default of the matrix
// it stands for, Copy follows to the earlier matrix it names (and that one's
// encoding is evaluated for type s).  False for a Copy that does not name an
// earlier matrix or an unknown mode.
bool resolve(int s, const DequantEncoding* enc, DequantEncoding* out) {
  int idx = s;
  while (true) {
    if (!enc || enc[idx].mode == kDqLibrary) {
      default_encoding(idx, out);
      return true;
    }
    const DequantEncoding& e = enc[idx];
    if (e.mode == kDqCopy) {
      if (e.copy_from < 0 || e.copy_from >= idx) return false;
      idx = e.copy_from;
      continue;
    }
    if (e.mode < kDqIdentity || e.mode > kDqDct) return false;
    *out = e;
    return true;
  }
}

}  // namespace

void default_encoding(int s, DequantEncoding* e) {
  std::memset(e, 0, sizeof(*e));
  switch (s) {
    case 1:
      e->mode = kDqIdentity;
      for (int c = 0; c < 3; ++c)
        for (int i = 0; i < 3; ++i) e->params[c][i] = kIdentityW[c][i];
      break;
    case 2:
      e->mode = kDqDct2;
      for (int c = 0; c < 3; ++c)
        for (int i = 0; i < 6; ++i) e->params[c][i] = kDct2W[c][i];
      break;
    case 3:
      e->mode = kDqDct4;
      set_bands(e, kDist4, nullptr, 2);
      for (int c = 0; c < 3; ++c)
        for (int i = 0; i < 2; ++i) e->params[c][i] = kDct4Mul[c][i];
      break;
    case 12:
    case 13:
      e->mode = kDqDct4x8;
      set_bands(e, kDist4x8, nullptr, 2);
      for (int c = 0; c < 3; ++c) e->params[c][0] = kDct4x8Mul[c];
      break;
    case 14:
      e->mode = kDqAfv;
      for (int c = 0; c < 3; ++c) {
        for (int i = 0; i < 8; ++i) e->afv_weights[c][i] = kAfvW[c][i];
        for (int i = 0; i < 2; ++i) e->params[c][i] = kAfvMul[c][i];
      }
      break;
    default:
      e->mode = kDqDct;
      switch (s) {
        case 0: set_bands(e, kDist8, nullptr, 3); break;
        case 4: set_bands(e, kDist16, nullptr, 3); break;
        case 5: set_bands(e, kDist32, nullptr, 4); break;
        case 6: case 7: set_bands(e, kDist16x8, nullptr, 3); break;
        case 8: case 9: set_bands(e, kDist32x8, &kEcc32x8, 4); break;
        default: set_bands(e, kDist32x16, nullptr, 4); break;
      }
      break;
  }
}

int dq_offset(int s) {
  int off = 0;
  for (int t = 0; t < s; ++t) off += 3 * 64 * blocks_x(t) * blocks_y(t);
  return off;
}

bool dequant_matrix_f64(int s, int c, double* out, const DequantEncoding* enc) {
  const int X = 8 * blocks_x(s), Y = 8 * blocks_y(s);
  DequantEncoding e;
  if (!resolve(s, enc, &e)) return false;
  // the Identity, DCT2, DCT4, DCT4x8 and AFV modes define 64-entry matrices only
  if (e.mode != kDqDct && X * Y != 64) return false;
  if ((e.mode == kDqDct || e.mode == kDqDct4 || e.mode == kDqDct4x8) &&
      (e.num_bands < 2 || e.num_bands > 17 || e.num_ecc_bands < 1 || e.num_ecc_bands > 8))
    return false;
  std::vector<double> w(size_t(X) * Y, 1.0), num(size_t(X) * Y, 1.0);
  auto at = [X](std::vector<double>& m, int x, int y) -> double& { return m[size_t(y) * X + x]; };
  const double* prm = e.params[c];
  const double* db = e.dist_bands[c];
  const double* eb = e.ecc_bands[c];
  switch (e.mode) {
    case kDqIdentity: {
      for (auto& v : w) v = prm[0];
      at(w, 1, 0) = at(w, 0, 1) = prm[1];
      at(w, 1, 1) = prm[2];
      break;
    }
    case kDqDct2: {  // index by the larger and smaller coordinate
      for (int y = 0; y < 8; ++y)
        for (int x = 0; x < 8; ++x) {
          const int hi = std::max(x, y), lo = std::min(x, y);
          int k = -1;
          if (hi == 1) k = lo;                 // (0,1)/(1,0) -> 0, (1,1) -> 1
          else if (hi >= 2 && hi < 4) k = lo < 2 ? 2 : 3;
          else if (hi >= 4) k = lo < 4 ? 4 : 5;
          if (k >= 0) at(w, x, y) = prm[k];
        }
      break;
    }
    case kDqDct4x8: {  // 8x4 band matrix at (x, y / 2); transposed for DCT8x4
      std::vector<double> w84 = band_weights(8, 4, db, e.num_bands, eb, e.num_ecc_bands);
      for (int y = 0; y < 8; ++y)
        for (int x = 0; x < 8; ++x) {
          const int u = s == 13 ? y : x, v = s == 13 ? x : y;  // the 8x4 matrix's column, row
          double wv = w84[(v / 2) * 8 + u];
          if (u == 0 && v == 1) wv /= prm[0];
          at(w, x, y) = wv;
        }
      break;
    }
    case kDqAfv: {  // 4x4 values, each covering a 2x2 cell group
      const double* aw = e.afv_weights[c];
      std::vector<double> bands = cumulative(aw[4], aw + 5, 3);
      double w4[16];
      w4[0] = aw[0];
      w4[4] = aw[1];  // group (0, 1)
      w4[1] = aw[2];  // group (1, 0)
      w4[5] = aw[3];
      for (int i = 0; i < 16; ++i)
        if ((i & 3) >= 2 || i >= 8) w4[i] = interp(kAfvFreq[i] - kAfvLo, kAfvHi, bands);
      for (int y = 0; y < 8; ++y)
        for (int x = 0; x < 8; ++x) at(w, x, y) = w4[(y / 2) * 4 + x / 2];
      at(w, 1, 0) *= prm[0];
      at(w, 0, 1) *= prm[0];
      at(w, 1, 1) *= prm[1];
      break;
    }
    case kDqDct4: {  // 4x4 band matrix, each entry covering 2x2
      std::vector<double> w4 = band_weights(4, 4, db, e.num_bands, eb, e.num_ecc_bands);
      for (int y = 0; y < 8; ++y)
        for (int x = 0; x < 8; ++x) at(w, x, y) = w4[(y / 2) * 4 + x / 2];
      at(w, 1, 0) /= prm[0];
      at(w, 0, 1) /= prm[0];
      at(w, 1, 1) /= prm[1];
      break;
    }
    default:  // DCT mode, the varblock's own size
      w = band_weights(X, Y, db, e.num_bands, eb, e.num_ecc_bands);
      break;
  }
  // Numerators by transform type: 1 for Identity, DCT2 and AFV; otherwise
  // I(N, f) per axis over X Y, with N = 4 and f = pos / 2 on an axis of
  // 4-point transforms.
  for (int y = 0; y < Y; ++y)
    for (int x = 0; x < X; ++x) {
      double v = 1.0;
      if (s == 3) v = scale_i(4, x / 2) * scale_i(4, y / 2) / 64.0;
      else if (s == 12) v = scale_i(8, x) * scale_i(4, y / 2) / 64.0;
      else if (s == 13) v = scale_i(4, x / 2) * scale_i(8, y) / 64.0;
      else if (s != 1 && s != 2 && s != 14) v = scale_i(X, x) * scale_i(Y, y) / (double(X) * Y);
      at(num, x, y) = v;
    }
  for (int i = 0; i < X * Y; ++i) {
    const double v = num[i] / w[i];
    if (i > 0 && !(v > 0.0 && std::isfinite(v))) return false;
    out[i] = v;
  }
  return true;
}

double transform_scale(int n, int k) {
  // T_N[r][k] = q_N[r][k] / I(N, k) and q_N = sqrt(eps_k / N) cos(...)
  return std::sqrt((k == 0 ? 1.0 : 2.0) / n) / scale_i(n, k);
}

void inverse_transform_matrix_f64(int n, double* out) {
  for (int r = 0; r < n; ++r)
    for (int k = 0; k < n; ++k) out[r * n + k] = ortho(n, r, k) / scale_i(n, k);
}

// J.2.4: Weight(sad, mul) as binary32 bits; mul <= 0.
static float epf_weight(int32_t sad, int32_t mul) {
  const int64_t pre = int64_t(sad < 507 ? sad : 507) << 6;
  const int64_t prod = pre * mul;
  // floor division by 2^16 (prod <= 0)
  const int64_t hi = (prod >= 0 ? prod / 65536 : -((-prod + 65535) / 65536)) + (127 << 7);
  const uint32_t bits = uint32_t(hi) << 16;
  float f;
  std::memcpy(&f, &bits, 4);
  return f;
}

void epf_mul_table(int sigma_shift, int32_t* table) {
  std::memset(table, 0, sizeof(int32_t) * 673);
  int32_t mul = -32768;
  for (int sigma = 16; sigma <= 672; sigma += 4) {
    while (mul < 0 && !(epf_weight(sigma >> sigma_shift, mul) > 0.5f)) ++mul;
    table[sigma] = mul;
  }
  // Between the computed points the step is truncated toward zero.
  for (int sigma = 16; sigma < 672; sigma += 4) {
    const int32_t step = (table[sigma + 4] - table[sigma]) / 4;
    for (int i = 1; i < 4; ++i) table[sigma + i] = table[sigma] + i * step;
  }
}

bool srgb_bucket_starts(uint8_t* start) {
  std::memset(start, 0, kSrgbBucketsPadded);
  for (int b = 0; b < kSrgbBuckets; ++b) {
    // smallest and largest binary32 value of the bucket (bucket 0 from 0)
    const uint32_t lo_bits = b == 0 ? 0u : uint32_t(kSrgbBucket0 + b) << 16;
    const uint32_t hi_bits = b == kSrgbBuckets - 1 ? lo_bits : (uint32_t(kSrgbBucket0 + b + 1) << 16) - 1;
    float lo, hi;
    std::memcpy(&lo, &lo_bits, 4);
    std::memcpy(&hi, &hi_bits, 4);
    const int c0 = srgb_code_f64(8, lo), c1 = srgb_code_f64(8, hi);
    if (c1 - c0 > 1) return false;
    start[b] = uint8_t(c0);
  }
  return true;
}

int srgb_code_f64(int bits, float v) {
  // IEC 61966-2-1 encoding of the clamped linear value, then round half up
  const double maxv = double((1 << bits) - 1);
  double x = double(v);
  x = x < 0.0 ? 0.0 : (x > 1.0 ? 1.0 : x);
  const double e = x <= 0.0031308 ? 12.92 * x : 1.055 * std::pow(x, 1.0 / 2.4) - 0.055;
  return int(std::floor(e * maxv + 0.5));
}

void srgb_thresholds(int bits, float* thr) {
  const int maxv = (1 << bits) - 1;
  thr[0] = -std::numeric_limits<float>::infinity();
  thr[maxv + 1] = std::numeric_limits<float>::infinity();
  for (int k = 1; k <= maxv; ++k) {
    // start at the binary64 inverse of the boundary (k - 0.5) / maxv and walk
    // to the first float whose code reaches k; codes are monotone in v
    const double e = (k - 0.5) / maxv;
    const double lin = e <= 12.92 * 0.0031308 ? e / 12.92 : std::pow((e + 0.055) / 1.055, 2.4);
    float v = float(lin);
    while (srgb_code_f64(bits, v) >= k) v = std::nextafter(v, -1.0f);
    while (srgb_code_f64(bits, v) < k) v = std::nextafter(v, 2.0f);
    thr[k] = v;
  }
}


uint16_t f16_rne(double v) {
  // sign, then the magnitude as an integer count of the format's spacing at
  // its exponent (2^-24 for subnormals), rounded to nearest even
  const uint16_t sign = v < 0 ? 0x8000u : 0u;
  double a = std::fabs(v);
  if (a == 0.0) return sign;
  int e;
  std::frexp(a, &e);  // a = f 2^e, f in [0.5, 1)
  int ulp_exp = std::max(e - 11, -24);  // spacing 2^(e - 11) for normals
  double q = std::nearbyint(std::ldexp(a, -ulp_exp));  // ties to even (default mode)
  if (q >= 2048.0) {  // rounded up into the next binade
    q /= 2.0;
    ulp_exp += 1;
  }
  const int biased = ulp_exp + 25;  // exponent field of a normal with this spacing
  if (q < 1024.0) return uint16_t(sign | uint16_t(q));  // subnormal (ulp_exp == -24)
  return uint16_t(sign | uint16_t(biased << 10) | (uint16_t(q) & 0x3FFu));
}

double f16_value(uint16_t h) {
  const int ex = (h >> 10) & 31, m = h & 1023;
  const double v = ex ? std::ldexp(1024.0 + m, ex - 25) : std::ldexp(double(m), -24);
  return (h & 0x8000u) ? -v : v;
}

namespace {
void build_mfma_operands(DeviceTables* t) {
  const double pi = 3.14159265358979323846;
  for (int m = 0; m < 3; ++m) {
    const int N = 8 << m;
    for (int step = 0; step < 2; ++step)
      for (int l = 0; l < 64; ++l)
        for (int e = 0; e < 8; ++e) {
          const int i = l % 32, k = 16 * step + 8 * (l / 32) + e;
          const double a = i / N == k / N ? std::cos(pi * (2 * (i % N) + 1) * (k % N) / (2.0 * N)) : 0.0;
          const uint16_t hh = f16_rne(16.0 * a);
          t->mfma_h[m][0][step][l][e] = hh;
          t->mfma_h[m][1][step][l][e] = f16_rne(16.0 * a - f16_value(hh));
        }
    for (int n = 0; n < 32; ++n)
      for (int u = 0; u < 4; ++u)
        t->llf_cos[m][n][u] =
            n < N && u < N / 8 ? float(std::cos(pi * (2 * n + 1) * u / (2.0 * N))) : 0.0f;
    for (int n = 0; n < 32; ++n)
      t->llf_c1[m][n] = n < N ? float(std::cos(pi * (2 * n + 1) / (2.0 * N))) : 0.0f;
  }
}
}  // namespace

bool build_tables(DeviceTables* t, const DequantEncoding* enc) {
  std::memset(t, 0, sizeof(*t));
  std::vector<double> m(32 * 32);
  inverse_transform_matrix_f64(8, m.data());
  for (int i = 0; i < 64; ++i) t->t8[i] = float(m[i]);
  inverse_transform_matrix_f64(16, m.data());
  for (int i = 0; i < 256; ++i) t->t16[i] = float(m[i]);
  inverse_transform_matrix_f64(32, m.data());
  for (int i = 0; i < 1024; ++i) t->t32[i] = float(m[i]);
  inverse_transform_matrix_f64(4, m.data());
  for (int half = 0; half < 2; ++half)
    for (int j = 0; j < 4; ++j)
      for (int i = 0; i < 4; ++i) t->m4[(4 * half + j) * 8 + half + 2 * i] = float(m[j * 4 + i]);
  // LLF from DC along one axis of a side with n DC samples (n = 2, 4):
  // a[x][i] = F_n[x][i] * ScaleF(n, 8 n, x) / n with the forward transform
  // F_n = n diag(I(n, .)) Q_n^T.
  for (int n : {2, 4}) {
    float* a = n == 2 ? t->a16 : t->a32;
    float* as = n == 2 ? t->a16s : t->a32s;
    for (int x = 0; x < n; ++x)
      for (int i = 0; i < n; ++i) {
        const double v = scale_i(n, x) * ortho(n, i, x) * scale_f(n, 8 * n, x);
        a[x * n + i] = float(v);
        as[x * n + i] = float(v * transform_scale(8 * n, x));
      }
  }
  // b = a^-1 for the scaled LLF-from-DC axis maps (Gauss-Jordan, partial
  // pivoting, in double from the double-precision entries).
  for (int n : {2, 4}) {
    double a[4][8] = {};
    for (int x = 0; x < n; ++x) {
      for (int i = 0; i < n; ++i)
        a[x][i] = scale_i(n, x) * ortho(n, i, x) * scale_f(n, 8 * n, x) * transform_scale(8 * n, x);
      a[x][n + x] = 1.0;
    }
    for (int col = 0; col < n; ++col) {
      int piv = col;
      for (int r = col + 1; r < n; ++r)
        if (std::fabs(a[r][col]) > std::fabs(a[piv][col])) piv = r;
      if (!(std::fabs(a[piv][col]) > 0.0)) return false;
      for (int j = 0; j < 2 * n; ++j) std::swap(a[col][j], a[piv][j]);
      const double d = a[col][col];
      for (int j = 0; j < 2 * n; ++j) a[col][j] /= d;
      for (int r = 0; r < n; ++r)
        if (r != col) {
          const double f = a[r][col];
          for (int j = 0; j < 2 * n; ++j) a[r][j] -= f * a[col][j];
        }
    }
    float* b = n == 2 ? t->b16s : t->b32s;
    for (int i = 0; i < n; ++i)
      for (int x = 0; x < n; ++x) b[i * n + x] = float(a[i][n + x]);
  }
  // AC prediction maps, one axis of 8 n pixels.  The side decoded from its
  // lowest coefficients (the inverse matrix T_N, N = 8 n) is averaged over
  // 4-pixel cells: W[j][k] = mean of T_N[4 j .. 4 j + 3][k], k < 2 n.  Cells
  // from DC: U = W[:, :n] A with A the LLF-from-DC axis map (1 for n = 1).
  // Coefficients from cells: V = W^-1 (Gauss-Jordan), rows scaled by s_N(k).
  for (int m = 0; m < 3; ++m) {
    const int n = 1 << m, N = 8 * n, c2 = 2 * n;
    std::vector<double> T(N * N);
    inverse_transform_matrix_f64(N, T.data());
    double W[8][16] = {};
    for (int j = 0; j < c2; ++j)
      for (int k = 0; k < c2; ++k) {
        double acc = 0.0;
        for (int r = 0; r < 4; ++r) acc += T[(4 * j + r) * N + k];
        W[j][k] = acc / 4.0;
      }
    for (int j = 0; j < c2; ++j)
      for (int i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int k = 0; k < n; ++k) {
          const double a = n == 1 ? 1.0 : scale_i(n, k) * ortho(n, i, k) * scale_f(n, 8 * n, k);
          acc += W[j][k] * a;
        }
        t->pred_u[m][j][i] = float(acc);
      }
    for (int j = 0; j < c2; ++j) W[j][c2 + j] = 1.0;
    for (int col = 0; col < c2; ++col) {
      int piv = col;
      for (int r = col + 1; r < c2; ++r)
        if (std::fabs(W[r][col]) > std::fabs(W[piv][col])) piv = r;
      if (!(std::fabs(W[piv][col]) > 0.0)) return false;
      for (int j = 0; j < 2 * c2; ++j) std::swap(W[col][j], W[piv][j]);
      const double d = W[col][col];
      for (int j = 0; j < 2 * c2; ++j) W[col][j] /= d;
      for (int r = 0; r < c2; ++r)
        if (r != col) {
          const double f = W[r][col];
          for (int j = 0; j < 2 * c2; ++j) W[r][j] -= f * W[col][j];
        }
    }
    for (int k = 0; k < c2; ++k)
      for (int j = 0; j < c2; ++j) t->pred_v[m][k][j] = float(W[k][c2 + j] * transform_scale(N, k));
  }
  // The generator step on the state (a, b) (first, second word):
  // a' = b, b' = u ^ b ^ (u >> 18) ^ (b >> 5) with u = a ^ (a << 23).  Its
  // matrix by columns (images of the unit states), then squared 13 times.
  {
    auto step = [](uint64_t a, uint64_t b, uint64_t& na, uint64_t& nb) {
      const uint64_t u = a ^ (a << 23);
      na = b;
      nb = u ^ b ^ (u >> 18) ^ (b >> 5);
    };
    // m[r][w]: row r, 128 bits in two words
    uint64_t m[128][2] = {};
    for (int j = 0; j < 128; ++j) {
      const uint64_t a = j < 64 ? uint64_t(1) << j : 0, b = j < 64 ? 0 : uint64_t(1) << (j - 64);
      uint64_t na, nb;
      step(a, b, na, nb);
      for (int r = 0; r < 128; ++r) {
        const uint64_t bit = r < 64 ? (na >> r) & 1u : (nb >> (r - 64)) & 1u;
        if (bit) m[r][j >> 6] |= uint64_t(1) << (j & 63);
      }
    }
    for (int k = 0; k < 14; ++k) {
      // column j of m (the image of unit state j), then the XOR of the
      // columns of each nibble value
      uint64_t col[128][2] = {};
      for (int r = 0; r < 128; ++r)
        for (int j = 0; j < 128; ++j)
          if ((m[r][j >> 6] >> (j & 63)) & 1u) col[j][r >> 6] |= uint64_t(1) << (r & 63);
      for (int p = 0; p < 32; ++p)
        for (int v = 0; v < 16; ++v) {
          uint64_t w0 = 0, w1 = 0;
          for (int b = 0; b < 4; ++b)
            if ((v >> b) & 1) {
              w0 ^= col[4 * p + b][0];
              w1 ^= col[4 * p + b][1];
            }
          t->noise_nib[k][p][v][0] = w0;
          t->noise_nib[k][p][v][1] = w1;
        }
      // m = m * m over GF(2): row r of the product is the XOR of the rows j
      // of m selected by the bits of row r
      uint64_t sq[128][2] = {};
      for (int r = 0; r < 128; ++r)
        for (int j = 0; j < 128; ++j)
          if ((m[r][j >> 6] >> (j & 63)) & 1u) {
            sq[r][0] ^= m[j][0];
            sq[r][1] ^= m[j][1];
          }
      std::memcpy(m, sq, sizeof(m));
    }
  }
  t->pred_sf = float(scale_f(2, 8, 1));
  t->pred_s8_1 = float(transform_scale(8, 1));
  for (int k = 0; k < 32; ++k)
    t->spline_scale[k] = scale_d(32, k) * (k == 0 ? 1.0 / (4.0 * std::sqrt(2.0)) : 0.25);
  {
    double t8[64];
    inverse_transform_matrix_f64(8, t8);
    for (int y = 0; y < 8; ++y)
      for (int u = 0; u < 8; ++u) t->jpeg1_a[y][u] = float(t8[y * 8 + u] * scale_i(8, u));
  }
  build_mfma_operands(t);
  for (int j = 0; j < 16; ++j)
    for (int i = 0; i < 16; ++i) t->afv[j][i] = float(kAfvBasis[j][i]);
  srgb_thresholds(8, t->srgb_thr8);
  srgb_thresholds(16, t->srgb_thr16);
  if (!srgb_bucket_starts(t->srgb_start8)) return false;
  std::vector<double> dq(1024);
  for (int s = 0; s < kNumStrategies; ++s) {
    const int X = 8 * blocks_x(s), Y = 8 * blocks_y(s), sz = X * Y;
    for (int c = 0; c < 3; ++c) {
      if (!dequant_matrix_f64(s, c, dq.data(), enc)) return false;
      for (int i = 0; i < sz; ++i) {
        const int x = i % X, y = i / X;
        double sc = 1.0;
        if (s == 3) sc = transform_scale(4, y / 2) * transform_scale(4, x / 2);
        else if (s == 12) sc = transform_scale(4, y / 2) * transform_scale(8, x);
        else if (s == 13) sc = transform_scale(8, y) * transform_scale(4, x / 2);
        else if (s == 14) sc = 1.0;
        else if (s != 1 && s != 2) sc = transform_scale(Y, y) * transform_scale(X, x);
        t->dq[dq_offset(s) + c * sz + i] = float(dq[i]);
        t->dqs[dq_offset(s) + c * sz + i] = float(dq[i] * sc);
      }
    }
  }
  for (int shift = 0; shift <= 8; ++shift) epf_mul_table(shift, t->mul_table[shift]);
  return true;
}

}  // namespace jxlr
