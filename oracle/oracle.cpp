/*
 * CPU ORACLE for the per-CTU coding-tree search -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is the plain, slow, obviously-correct definition that the GPU
 * library is checked against.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header, table
 * or constant generator with the GPU library; it is compiled by gcc alone.
 *
 * What it computes (thesis sections cited; readings where the thesis is
 * silent are marked READING):
 *   - CTU of 64x64 luma split by a quad-tree into CUs 64, 32, 16, 8
 *     (HEVC background section: CTB sizes, CU quad-tree 8x8..64x64).
 *   - Rate-distortion choice over partitions and modes (HEVC background
 *     section: RDO over the quad-tree), with costs J = D + sqrt(lambda) * R
 *     kept as integers in Q16: J = D * 65536 + s * R, s = round(sqrt(lambda)*65536).
 *     READING: lambda = 0.57 * 2^((QP-12)/3) (the HM convention; the thesis
 *     gives no lambda).
 *   - SAD (cost-function subsection, first equation) for integer-pel full
 *     search motion estimation; the ME cost adds sqrt(lambda) times the
 *     signed Exp-Golomb length of the quarter-pel MV components, predictor
 *     (0,0).  READING: all (2R+1)^2 candidates, reference samples clamped to
 *     the picture, first strict minimum in raster order (dy outer, dx inner).
 *   - SATD (cost-function subsection, second equation): sum of |H| / 2 with
 *     H the 4x4 Hadamard transform of the residual, tiles aligned to the CU
 *     origin.  The thesis's C++ SATD listing works on 4x4 Hadamard tiles (two
 *     at a time, halved once per pair); every 4x4 sum of |H| is even, so the
 *     per-tile halving used here is the same number.
 *   - Intra DC and planar (HEVC background section names DC/planar/angular;
 *     formulas are the H.265 ones) from original neighbouring samples.
 *     READING: a neighbour is available iff it lies inside the coded picture;
 *     H.265 reference substitution; no reference smoothing, no DC edge filter.
 *   - Optionally the 33 angular modes (same section), H.265 angular
 *     prediction from the same substituted neighbours.  READING: no
 *     reference smoothing and no edge filter for the pure horizontal and
 *     vertical modes (as for DC); mode bits from the H.265 most-probable-mode
 *     list of a block whose neighbours are unavailable, {planar, DC,
 *     vertical}: 1 (prediction mode) + 1 (MPM flag) + 1 or 2 (MPM index) for
 *     planar (3), DC (4) and vertical (4), 1 + 1 + 5 (fixed-length remainder)
 *     = 7 for the other 32; ties in the order inter < planar < DC < angular by
 *     mode number.  Mode codes: 0 inter, 1 + the H.265 intra mode otherwise.
 *   - Bottom-up quad-tree decision with optional per-8x8 depth bounds; the
 *     bounds implement depth-bound reuse (related-work section: search only
 *     depths up to the co-located reference depth) generalised to scaled
 *     resolutions (related-work section: arbitrary down-sampling ratio; x265
 *     scale-factor option in the analysis-share appendix; refine-intra level 1
 *     "depth n and n+1" in the analysis-refinement appendix).
 *
 *   - Seeded search (motion-vector reuse with refinement, the x265 refine-mv
 *     option of the analysis-refinement appendix; the reuse of reference MVs
 *     at scaled resolutions in the related-work section).  READING (the
 *     thesis's MV-refinement table is empty): every CU takes the MV of the
 *     reference unit co-located with its centre, scales it by the width and
 *     height ratios (rounded half away from zero), clamps it to
 *     [-(R - r), R - r] and searches the (2r+1)^2 displacements around it
 *     with the same cost and tie order as the full search.  r = R is the
 *     full search.
 *   - Sub-pel refinement (SATD for quarter-pel motion estimation, cost-function
 *     subsection; interpolation filters among the thesis's optimised
 *     functions).  READING: H.265 8-bit luma fractional interpolation with the
 *     default uni-prediction rounding; after the integer ME, a half-pel stage
 *     and a quarter-pel stage, each over the current best and its 8
 *     neighbours, J = SATD * 65536 + s * (se(qx) + se(qy)) in quarter-pel
 *     units, ties to the centre then raster order; MVs are then output in
 *     quarter-pel units.
 *
 * No blocking, fusion or reordering: SAD is summed directly per CU and per
 * candidate; the DP is a plain recursion.
 */
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <thread>
#include <vector>

namespace {

constexpr int kCtu = 64;

struct Pic {
  const uint8_t* p;
  int w, h, stride;
  int w8, h8;  // coded size: multiples of 8 (HEVC minimum CU), edge-replicated
};

Pic make_pic(const uint8_t* p, int w, int h, int stride) {
  Pic c{p, w, h, stride, (w + 7) / 8 * 8, (h + 7) / 8 * 8};
  return c;
}

// Coded picture sample C(x, y), 0 <= x < w8, 0 <= y < h8 (padding by edge replication).
inline int coded(const Pic& c, int x, int y) {
  return c.p[(int64_t)std::min(y, c.h - 1) * c.stride + std::min(x, c.w - 1)];
}

// Reference sample at any integer position, coordinates clamped to the picture.
inline int refs(const Pic& r, int x, int y) {
  x = std::min(std::max(x, 0), r.w - 1);
  y = std::min(std::max(y, 0), r.h - 1);
  return r.p[(int64_t)y * r.stride + x];
}

int64_t sqrt_lambda_q16(int qp) {
  double lambda = 0.57 * std::pow(2.0, (qp - 12) / 3.0);
  return (int64_t)std::llround(std::sqrt(lambda) * 65536.0);
}

// Number of bits of the signed Exp-Golomb code se(v): v maps to codeNum
// k = 2v-1 (v>0) or -2v (v<=0); ue(k) has 2*floor(log2(k+1)) + 1 bits.
int se_bits(int v) {
  int64_t k = v > 0 ? 2 * (int64_t)v - 1 : -2 * (int64_t)v;
  int64_t m = k + 1;
  int lg = 0;
  while (m > 1) {
    m >>= 1;
    ++lg;
  }
  return 2 * lg + 1;
}

int mv_bits(int mx, int my) { return se_bits(4 * mx) + se_bits(4 * my); }

// SATD of one 4x4 residual tile: sum |Hd * D * Hd^T| / 2 by plain matrix products.
int64_t satd4(const int d[4][4]) {
  static const int Hd[4][4] = {{1, 1, 1, 1}, {1, -1, 1, -1}, {1, 1, -1, -1}, {1, -1, -1, 1}};
  int t[4][4], u[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      int s = 0;
      for (int k = 0; k < 4; ++k) s += Hd[i][k] * d[k][j];
      t[i][j] = s;
    }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      int s = 0;
      for (int k = 0; k < 4; ++k) s += t[i][k] * Hd[j][k];
      u[i][j] = s;
    }
  int64_t sum = 0;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) sum += std::abs(u[i][j]);
  return sum / 2;
}

// SATD of an n x n residual (n multiple of 4): sum over 4x4 tiles aligned to the origin.
int64_t satd_block(const int* resid, int stride, int n) {
  int64_t total = 0;
  for (int ty = 0; ty < n; ty += 4)
    for (int tx = 0; tx < n; tx += 4) {
      int d[4][4];
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) d[i][j] = resid[(ty + i) * stride + tx + j];
      total += satd4(d);
    }
  return total;
}

// H.265 intraPredAngle of intra modes 2..34 (index = mode), and invAngle of
// the modes with a negative angle (11..25): 8192 / angle rounded to nearest.
const int kIntraAngle[35] = {0,   0,   32,  26,  21,  17,  13,  9,   5,   2,   0,   -2,
                             -5,  -9,  -13, -17, -21, -26, -32, -26, -21, -17, -13, -9,
                             -5,  -2,  0,   2,   5,   9,   13,  17,  21,  26,  32};
int inv_angle(int angle) {
  switch (angle) {
    case -2: return -4096;
    case -5: return -1638;
    case -9: return -910;
    case -13: return -630;
    case -17: return -482;
    case -21: return -390;
    case -26: return -315;
    case -32: return -256;
    default: return 0;
  }
}

// Intra prediction (mode code 1 planar, 2 DC, 1 + m for the angular mode m in
// 2..34) of the n x n block at (x0, y0) of the coded current picture.
// Neighbours: left column p[-1][y], y = -1..2n-1 (corner included) and top
// row p[x][-1], x = 0..2n-1.
void intra_predict(const Pic& c, int x0, int y0, int n, int mode, int* pred) {
  std::vector<int> left(2 * n + 1), top(2 * n);  // left[y + 1] = p[-1][y]
  std::vector<char> lav(2 * n + 1), tav(2 * n);
  auto inside = [&](int x, int y) { return x >= 0 && y >= 0 && x < c.w8 && y < c.h8; };
  bool any = false;
  for (int y = -1; y < 2 * n; ++y) {
    lav[y + 1] = inside(x0 - 1, y0 + y);
    if (lav[y + 1]) left[y + 1] = coded(c, x0 - 1, y0 + y), any = true;
  }
  for (int x = 0; x < 2 * n; ++x) {
    tav[x] = inside(x0 + x, y0 - 1);
    if (tav[x]) top[x] = coded(c, x0 + x, y0 - 1), any = true;
  }
  if (!any) {
    std::fill(left.begin(), left.end(), 128);
    std::fill(top.begin(), top.end(), 128);
  } else {
    // Substitution: the bottom-left sample takes the first available value
    // found scanning up the left column, then along the top row.
    if (!lav[2 * n]) {
      int v = -1;
      for (int y = 2 * n - 1; y >= -1 && v < 0; --y)
        if (lav[y + 1]) v = left[y + 1];
      for (int x = 0; x < 2 * n && v < 0; ++x)
        if (tav[x]) v = top[x];
      left[2 * n] = v;
      lav[2 * n] = 1;
    }
    for (int y = 2 * n - 2; y >= -1; --y)
      if (!lav[y + 1]) left[y + 1] = left[y + 2], lav[y + 1] = 1;
    for (int x = 0; x < 2 * n; ++x)
      if (!tav[x]) top[x] = (x == 0 ? left[0] : top[x - 1]), tav[x] = 1;
  }
  int lg = 0;
  while ((1 << lg) < n) ++lg;
  if (mode >= 3) {  // angular: H.265 mode m = mode - 1
    const int m = mode - 1, angle = kIntraAngle[m];
    const bool vertical = m >= 18;
    // main[k], k = 0..2n: the corner then the samples along the prediction's
    // own side (top row for vertical modes, left column for horizontal ones);
    // side[k] likewise along the other side.  left[k] = p[-1][k - 1].
    std::vector<int> main_(2 * n + 1), side(2 * n + 1);
    for (int k = 0; k <= 2 * n; ++k) {
      const int t = k == 0 ? left[0] : top[k - 1];
      const int l = left[k];
      main_[k] = vertical ? t : l;
      side[k] = vertical ? l : t;
    }
    // ref[k] for k = -n..2n at ref[k + n]: main for k >= 0; for a negative
    // angle reaching past the corner, the other side projected onto the main
    // line: ref[k] = side[(k * invAngle + 128) >> 8].
    std::vector<int> ref(3 * n + 1, 0);
    for (int k = 0; k <= 2 * n; ++k) ref[k + n] = main_[k];
    if (angle < 0 && ((n * angle) >> 5) < -1) {
      const int inv = inv_angle(angle);
      for (int k = (n * angle) >> 5; k <= -1; ++k) ref[k + n] = side[(k * inv + 128) >> 8];
    }
    for (int y = 0; y < n; ++y)
      for (int x = 0; x < n; ++x) {
        // Along the prediction direction: the row (vertical) or column
        // (horizontal) distance from the reference line, and the position
        // across it.
        const int along = vertical ? y : x, across = vertical ? x : y;
        const int pos = (along + 1) * angle;
        const int idx = pos >> 5, fact = pos & 31;
        const int a = ref[across + idx + 1 + n];
        pred[y * n + x] = fact ? ((32 - fact) * a + fact * ref[across + idx + 2 + n] + 16) >> 5 : a;
      }
    return;
  }
  if (mode == 1) {  // planar
    for (int y = 0; y < n; ++y)
      for (int x = 0; x < n; ++x)
        pred[y * n + x] = ((n - 1 - x) * left[y + 1] + (x + 1) * top[n] + (n - 1 - y) * top[x] +
                           (y + 1) * left[n + 1] + n) >>
                          (lg + 1);
  } else {  // DC
    int s = n;
    for (int x = 0; x < n; ++x) s += top[x];
    for (int y = 0; y < n; ++y) s += left[y + 1];
    int dc = s >> (lg + 1);
    for (int i = 0; i < n * n; ++i) pred[i] = dc;
  }
}

struct Node {
  int kind;  // 0 absent (outside the coded picture), 1 crosses its edge, 2 inside
  int mx, my;          // integer ME result
  int qmx, qmy;        // final MV in quarter-pel units (4 mx, 4 my without sub-pel refinement)
  int64_t sad;
  int64_t satd_inter, satd_planar, satd_dc;
  int64_t satd_angular_best;  // smallest SATD over the angular modes (-1: not evaluated)
  int mode;            // 0 inter, 1 planar, 2 DC, 3..35 angular (1 + H.265 mode)
  int64_t leaf_j;      // J of the best mode, without the split flag
  int64_t leaf_d, leaf_r;
  int evaluated;
};

// Integer ME for one CU over the square window of half-width R around
// (wx, wy): exhaustive over dy = wy-R..wy+R (outer), dx = wx-R..wx+R (inner);
// J = SAD * 65536 + s * (se(4dx) + se(4dy)); first strict minimum.  The full
// search is the window centred at (0, 0).
void cu_motion_search(const Pic& cur, const Pic& ref, int x0, int y0, int n, int wx, int wy,
                      int R, int64_t s, int* bmx, int* bmy, int64_t* bsad) {
  int64_t best = INT64_MAX;
  for (int dy = wy - R; dy <= wy + R; ++dy)
    for (int dx = wx - R; dx <= wx + R; ++dx) {
      int64_t sad = 0;
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i)
          sad += std::abs(coded(cur, x0 + i, y0 + j) - refs(ref, x0 + i + dx, y0 + j + dy));
      int64_t jme = sad * 65536 + s * mv_bits(dx, dy);
      if (jme < best) best = jme, *bmx = dx, *bmy = dy, *bsad = sad;
    }
}

// Reference MVs for a seeded search: the per-8x8 MV map of a search of the
// same content at another resolution (ref_w x ref_h), and the refinement
// half-width r.
struct Seed {
  const int16_t* ref_mv;  // [ceil(ref_h/8)][ceil(ref_w/8)][2]
  int ref_w, ref_h;
  int r;
  int qpel;  // 1: the map holds quarter-pel MVs (a search with sub-pel refinement)
};

// m * num / den rounded to the nearest integer, halves away from zero.
int scale_round(int m, int num, int den) {
  int64_t a = std::abs((int64_t)m) * num;
  int64_t q = (2 * a + den) / (2 * (int64_t)den);
  return (int)(m < 0 ? -q : q);
}

// Search centre of the n x n CU at (x0, y0) of a cur_w x cur_h picture: the
// reference unit co-located with the CU's centre sample (same mapping as the
// depth bounds), its MV scaled by the dimension ratios, clamped so that the
// window of half-width r stays inside [-R, R].
void mv_centre(const Seed& sd, int cur_w, int cur_h, int R, int x0, int y0, int n, int* cx,
               int* cy) {
  int64_t px = x0 + n / 2, py = y0 + n / 2;
  int64_t xr = std::min<int64_t>(px * sd.ref_w / cur_w, sd.ref_w - 1);
  int64_t yr = std::min<int64_t>(py * sd.ref_h / cur_h, sd.ref_h - 1);
  int ruw = (sd.ref_w + 7) / 8;
  const int16_t* m = sd.ref_mv + 2 * ((yr / 8) * ruw + xr / 8);
  int lim = R - sd.r;
  const int unit = sd.qpel ? 4 : 1;  // map units per pixel
  *cx = std::clamp(scale_round(m[0], cur_w, sd.ref_w * unit), -lim, lim);
  *cy = std::clamp(scale_round(m[1], cur_h, sd.ref_h * unit), -lim, lim);
}

// ------------------------------------------------------------- sub-pel motion
// H.265 luma fractional-sample interpolation for 8-bit samples, then the
// default (unweighted) uni-prediction rounding back to 8 bits.  Filter taps per
// quarter-pel phase (the standard's luma interpolation filter table).
const int kLumaTaps[4][8] = {{0, 0, 0, 64, 0, 0, 0, 0},
                             {-1, 4, -10, 58, 17, -5, 1, 0},
                             {-1, 4, -11, 40, 40, -11, 4, -1},
                             {0, 1, -5, 17, 58, -10, 4, -1}};

// Floor division of a quarter-pel coordinate into (integer, phase).
inline void qsplit(int q, int* i, int* f) {
  *f = q & 3;
  *i = (q - *f) / 4;
}

// Prediction sample at quarter-pel position (qx, qy) of the reference.
// Integer positions: the sample scaled by 64; one fractional axis: the 8-tap
// sum (no shift for 8-bit); both: horizontal sums, then the vertical 8-tap sum
// of those shifted right by 6 (arithmetic).  Last: (v + 32) >> 6, clipped.
int interp_qpel(const Pic& ref, int qx, int qy) {
  int xi, fx, yi, fy;
  qsplit(qx, &xi, &fx);
  qsplit(qy, &yi, &fy);
  int64_t v;
  if (fx == 0 && fy == 0) {
    v = (int64_t)refs(ref, xi, yi) << 6;
  } else if (fy == 0) {
    v = 0;
    for (int i = 0; i < 8; ++i) v += kLumaTaps[fx][i] * refs(ref, xi + i - 3, yi);
  } else if (fx == 0) {
    v = 0;
    for (int i = 0; i < 8; ++i) v += kLumaTaps[fy][i] * refs(ref, xi, yi + i - 3);
  } else {
    int64_t acc = 0;
    for (int j = 0; j < 8; ++j) {
      int64_t h = 0;
      for (int i = 0; i < 8; ++i) h += kLumaTaps[fx][i] * refs(ref, xi + i - 3, yi + j - 3);
      acc += kLumaTaps[fy][j] * h;
    }
    v = acc >> 6;  // arithmetic shift: floor
  }
  int64_t p = (v + 32) >> 6;
  return (int)std::min<int64_t>(255, std::max<int64_t>(0, p));
}

// SATD of the n x n CU at (x0, y0) against the prediction at quarter-pel MV (qmx, qmy).
int64_t satd_at_qpel(const Pic& cur, const Pic& ref, int x0, int y0, int n, int qmx, int qmy) {
  std::vector<int> resid(n * n);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i)
      resid[j * n + i] =
          coded(cur, x0 + i, y0 + j) - interp_qpel(ref, 4 * (x0 + i) + qmx, 4 * (y0 + j) + qmy);
  return satd_block(resid.data(), n, n);
}

// Sub-pel refinement of an integer MV: a half-pel stage (step 2) and a
// quarter-pel stage (step 1), each over the current best and its 8
// neighbours at the step; J = SATD * 65536 + s * (se(qx) + se(qy)) with the
// MV in quarter-pel units; the centre keeps ties, then raster order (dy outer).
void subpel_refine(const Pic& cur, const Pic& ref, int x0, int y0, int n, int mx, int my,
                   int64_t s, int* bqx, int* bqy, int64_t* bsatd) {
  int qx = 4 * mx, qy = 4 * my;
  int64_t sd = satd_at_qpel(cur, ref, x0, y0, n, qx, qy);
  int64_t best = sd * 65536 + s * (se_bits(qx) + se_bits(qy));
  for (int step = 2; step >= 1; --step) {
    const int cqx = qx, cqy = qy;
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        if (dx == 0 && dy == 0) continue;
        const int tx = cqx + step * dx, ty = cqy + step * dy;
        const int64_t t = satd_at_qpel(cur, ref, x0, y0, n, tx, ty);
        const int64_t j = t * 65536 + s * (se_bits(tx) + se_bits(ty));
        if (j < best) best = j, qx = tx, qy = ty, sd = t;
      }
  }
  *bqx = qx, *bqy = qy, *bsatd = sd;
}

void evaluate_leaf(const Pic& cur, const Pic& ref, int x0, int y0, int n, int R, int64_t s,
                   const Seed* seed, bool subpel, bool angular, Node* nd) {
  if (seed) {
    int cx, cy;
    mv_centre(*seed, cur.w, cur.h, R, x0, y0, n, &cx, &cy);
    cu_motion_search(cur, ref, x0, y0, n, cx, cy, seed->r, s, &nd->mx, &nd->my, &nd->sad);
  } else {
    cu_motion_search(cur, ref, x0, y0, n, 0, 0, R, s, &nd->mx, &nd->my, &nd->sad);
  }
  std::vector<int> resid(n * n), pred(n * n);
  if (subpel) {
    subpel_refine(cur, ref, x0, y0, n, nd->mx, nd->my, s, &nd->qmx, &nd->qmy, &nd->satd_inter);
  } else {
    nd->qmx = 4 * nd->mx, nd->qmy = 4 * nd->my;
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i)
        resid[j * n + i] =
            coded(cur, x0 + i, y0 + j) - refs(ref, x0 + i + nd->mx, y0 + j + nd->my);
    nd->satd_inter = satd_block(resid.data(), n, n);
  }
  for (int mode = 1; mode <= 2; ++mode) {
    intra_predict(cur, x0, y0, n, mode, pred.data());
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) resid[j * n + i] = coded(cur, x0 + i, y0 + j) - pred[j * n + i];
    (mode == 1 ? nd->satd_planar : nd->satd_dc) = satd_block(resid.data(), n, n);
  }
  // Mode bits: 1 (prediction mode) + MV bits (quarter-pel components) for
  // inter; planar 3, DC 4.
  int64_t r_inter = 1 + se_bits(nd->qmx) + se_bits(nd->qmy), r_pl = 3, r_dc = 4;
  int64_t j_inter = nd->satd_inter * 65536 + s * r_inter;
  int64_t j_pl = nd->satd_planar * 65536 + s * r_pl;
  int64_t j_dc = nd->satd_dc * 65536 + s * r_dc;
  nd->mode = 0, nd->leaf_j = j_inter, nd->leaf_d = nd->satd_inter, nd->leaf_r = r_inter;
  if (j_pl < nd->leaf_j) nd->mode = 1, nd->leaf_j = j_pl, nd->leaf_d = nd->satd_planar, nd->leaf_r = r_pl;
  if (j_dc < nd->leaf_j) nd->mode = 2, nd->leaf_j = j_dc, nd->leaf_d = nd->satd_dc, nd->leaf_r = r_dc;
  // Angular modes 2..34 (codes 3..35): 4 bits for vertical (26, an MPM), 7 for the others.
  nd->satd_angular_best = -1;
  if (angular) {
    for (int m = 2; m <= 34; ++m) {
      intra_predict(cur, x0, y0, n, m + 1, pred.data());
      for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) resid[j * n + i] = coded(cur, x0 + i, y0 + j) - pred[j * n + i];
      const int64_t sd = satd_block(resid.data(), n, n), r_a = m == 26 ? 4 : 7;
      const int64_t j_a = sd * 65536 + s * r_a;
      if (nd->satd_angular_best < 0 || sd < nd->satd_angular_best) nd->satd_angular_best = sd;
      if (j_a < nd->leaf_j) nd->mode = m + 1, nd->leaf_j = j_a, nd->leaf_d = sd, nd->leaf_r = r_a;
    }
  }
  nd->evaluated = 1;
}

// Node index within a CTU: depth offsets 0, 1, 5, 21; raster order inside a depth.
int node_index(int d, int lx, int ly) {
  static const int off[4] = {0, 1, 5, 21};
  return off[d] + ly * (1 << d) + lx;
}

struct CtuJob {
  const Pic* cur;
  const Pic* ref;
  int R;
  int64_t s;
  const uint8_t* bounds;  // [h8/8][w8/8][2] or null
  const Seed* seed;       // null for the full search
  bool subpel;            // half- and quarter-pel refinement of the inter MV
  bool angular;           // the 33 angular intra modes beside planar and DC
  int cx, cy;             // CTU origin in pixels
  Node nodes[85];
};

struct Result {
  int64_t j, d, r;
};

void node_bounds(const CtuJob& job, int x0, int y0, int n, int* min_lo, int* max_hi) {
  const Pic& c = *job.cur;
  int uw = c.w8 / 8;
  *min_lo = 3, *max_hi = 0;
  for (int y = y0; y < y0 + n && y < c.h8; y += 8)
    for (int x = x0; x < x0 + n && x < c.w8; x += 8) {
      const uint8_t* b = job.bounds + 2 * ((int64_t)(y / 8) * uw + x / 8);
      *min_lo = std::min(*min_lo, (int)b[0]);
      *max_hi = std::max(*max_hi, (int)b[1]);
    }
}

// Bottom-up decision for node (d, lx, ly): the cheapest admissible coding of
// the node (leaf with its best mode, or the sum of its four children).
Result best_tree(CtuJob& job, int d, int lx, int ly, bool* choose_leaf) {
  const Pic& c = *job.cur;
  int n = kCtu >> d;
  int x0 = job.cx + lx * n, y0 = job.cy + ly * n;
  Node& nd = job.nodes[node_index(d, lx, ly)];
  Result res{0, 0, 0};
  if (x0 >= c.w8 || y0 >= c.h8) {
    nd.kind = 0;
    *choose_leaf = false;
    return res;
  }
  auto children = [&]() {
    Result sum{0, 0, 0};
    for (int k = 0; k < 4; ++k) {
      bool leaf;
      Result r = best_tree(job, d + 1, 2 * lx + (k & 1), 2 * ly + (k >> 1), &leaf);
      sum.j += r.j, sum.d += r.d, sum.r += r.r;
    }
    return sum;
  };
  if (x0 + n > c.w8 || y0 + n > c.h8) {  // crosses the picture edge: implicit split
    nd.kind = 1;
    *choose_leaf = false;
    return children();
  }
  nd.kind = 2;
  bool split_ok = d < 3, leaf_ok = true;
  if (job.bounds) {
    int min_lo, max_hi;
    node_bounds(job, x0, y0, n, &min_lo, &max_hi);
    split_ok = d < 3 && d < max_hi;
    leaf_ok = d >= min_lo || !split_ok;
  }
  Result leaf{INT64_MAX, 0, 0};
  if (leaf_ok) {
    if (!nd.evaluated)
      evaluate_leaf(*job.cur, *job.ref, x0, y0, n, job.R, job.s, job.seed, job.subpel,
                    job.angular, &nd);
    int flag = d < 3 ? 1 : 0;
    leaf = Result{nd.leaf_j + job.s * flag, nd.leaf_d, nd.leaf_r + flag};
  }
  if (split_ok) {
    Result sp = children();
    sp.j += job.s, sp.r += 1;
    if (!leaf_ok || sp.j < leaf.j) {
      *choose_leaf = false;
      return sp;
    }
  }
  *choose_leaf = true;
  return leaf;
}

// Second pass: re-run the decision top-down and write the chosen leaves.
void write_tree(CtuJob& job, int d, int lx, int ly, uint8_t* depth_out, uint8_t* mode_out,
                int16_t* mv_out) {
  const Pic& c = *job.cur;
  int n = kCtu >> d;
  int x0 = job.cx + lx * n, y0 = job.cy + ly * n;
  if (x0 >= c.w8 || y0 >= c.h8) return;
  bool leaf = false;
  best_tree(job, d, lx, ly, &leaf);
  if (!leaf) {
    for (int k = 0; k < 4; ++k)
      write_tree(job, d + 1, 2 * lx + (k & 1), 2 * ly + (k >> 1), depth_out, mode_out, mv_out);
    return;
  }
  const Node& nd = job.nodes[node_index(d, lx, ly)];
  int uw = c.w8 / 8;
  for (int y = y0; y < y0 + n; y += 8)
    for (int x = x0; x < x0 + n; x += 8) {
      int64_t u = (int64_t)(y / 8) * uw + x / 8;
      depth_out[u] = (uint8_t)d;
      mode_out[u] = (uint8_t)nd.mode;
      // Integer-pel units, or quarter-pel units with sub-pel refinement.
      mv_out[2 * u] = (int16_t)(job.subpel ? nd.qmx : nd.mx);
      mv_out[2 * u + 1] = (int16_t)(job.subpel ? nd.qmy : nd.my);
    }
}

bool valid_pic(const uint8_t* p, int w, int h, int stride) {
  return p && w > 0 && h > 0 && stride >= w;
}

}  // namespace

extern "C" {

int64_t orc_sqrt_lambda_q16(int qp) { return sqrt_lambda_q16(qp); }
int orc_se_bits(int v) { return se_bits(v); }
int64_t orc_satd(const int32_t* resid, int stride, int n) {
  std::vector<int> r(n * n);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) r[j * n + i] = resid[j * stride + i];
  return satd_block(r.data(), n, n);
}

// Intra prediction of the n x n block at (x0, y0); mode 1 planar, 2 DC,
// 3..35 the angular mode (mode - 1).
int orc_intra_predict(const uint8_t* cur, int w, int h, int stride, int x0, int y0, int n,
                      int mode, int32_t* pred) {
  if (!valid_pic(cur, w, h, stride) || mode < 1 || mode > 35 || n < 4) return -1;
  Pic c = make_pic(cur, w, h, stride);
  std::vector<int> p(n * n);
  intra_predict(c, x0, y0, n, mode, p.data());
  for (int i = 0; i < n * n; ++i) pred[i] = p[i];
  return 0;
}

// Exhaustive ME of one CU; returns the MV and its SAD.
int orc_cu_motion_search(const uint8_t* cur, const uint8_t* ref, int w, int h, int stride,
                         int x0, int y0, int n, int R, int qp, int32_t* mx, int32_t* my,
                         int64_t* sad) {
  if (!valid_pic(cur, w, h, stride) || !ref || R < 0) return -1;
  Pic c = make_pic(cur, w, h, stride), r = make_pic(ref, w, h, stride);
  int a, b;
  int64_t sd;
  cu_motion_search(c, r, x0, y0, n, 0, 0, R, sqrt_lambda_q16(qp), &a, &b, &sd);
  *mx = a, *my = b, *sad = sd;
  return 0;
}

// Seed arguments shared by the entry points below: ref_mv null means full
// search; otherwise the reference MV map of a ref_w x ref_h picture and the
// refinement half-width r (0 <= r <= R).
static bool make_seed(const int16_t* ref_mv, int ref_w, int ref_h, int r, int R, int qpel,
                      Seed* sd) {
  if (!ref_mv) return true;
  if (ref_w <= 0 || ref_h <= 0 || r < 0 || r > R || qpel < 0 || qpel > 1) return false;
  *sd = Seed{ref_mv, ref_w, ref_h, r, qpel};
  return true;
}

// Interpolated prediction sample at quarter-pel position (qx, qy).
int orc_interp_qpel(const uint8_t* ref, int w, int h, int stride, int qx, int qy) {
  if (!valid_pic(ref, w, h, stride)) return -1;
  return interp_qpel(make_pic(ref, w, h, stride), qx, qy);
}

// Sub-pel refinement of the integer MV (mx, my) of one CU: quarter-pel MV and its SATD.
int orc_subpel_refine(const uint8_t* cur, const uint8_t* ref, int w, int h, int stride, int x0,
                      int y0, int n, int mx, int my, int qp, int32_t* qx, int32_t* qy,
                      int64_t* satd) {
  if (!valid_pic(cur, w, h, stride) || !ref || qp < 0 || qp > 51 || n < 4) return -1;
  Pic c = make_pic(cur, w, h, stride), r = make_pic(ref, w, h, stride);
  int a, b;
  int64_t sd;
  subpel_refine(c, r, x0, y0, n, mx, my, sqrt_lambda_q16(qp), &a, &b, &sd);
  *qx = a, *qy = b, *satd = sd;
  return 0;
}

// Search centre of one CU for a seeded search (see mv_centre).
int orc_mv_centre(const int16_t* ref_mv, int ref_w, int ref_h, int cur_w, int cur_h, int R,
                  int r, int qpel, int x0, int y0, int n, int32_t* cx, int32_t* cy) {
  Seed sd{};
  if (!ref_mv || cur_w <= 0 || cur_h <= 0 ||
      !make_seed(ref_mv, ref_w, ref_h, r, R, qpel, &sd))
    return -1;
  int a, b;
  mv_centre(sd, cur_w, cur_h, R, x0, y0, n, &a, &b);
  *cx = a, *cy = b;
  return 0;
}

// Per-node leaf evaluation of one CTU (all 85 nodes, no bounds); record layout
// per node: kind, mode, mx, my, sad, satd_inter, satd_planar, satd_dc, leaf_j,
// leaf_d, leaf_r, qmx, qmy, satd_angular_best (14 int64; mx, my integer ME,
// qmx, qmy the final MV in quarter-pel units).  Used to check the decision
// against enumeration.  flags: bit 0 sub-pel refinement, bit 1 angular modes.
int orc_ctu_nodes(const uint8_t* cur, const uint8_t* ref, int w, int h, int stride, int qp,
                  int R, int flags, int ctu_x, int ctu_y, const int16_t* ref_mv, int ref_w,
                  int ref_h, int refine_r, int seed_qpel, int64_t* rec) {
  Seed sd{};
  if (!valid_pic(cur, w, h, stride) || !ref || R < 0 || qp < 0 || qp > 51 || flags < 0 ||
      flags > 3 || !make_seed(ref_mv, ref_w, ref_h, refine_r, R, seed_qpel, &sd))
    return -1;
  const bool subpel = (flags & 1) != 0, angular = (flags & 2) != 0;
  Pic c = make_pic(cur, w, h, stride), r = make_pic(ref, w, h, stride);
  CtuJob* job = new CtuJob();
  job->cur = &c, job->ref = &r, job->R = R, job->s = sqrt_lambda_q16(qp), job->bounds = nullptr;
  job->seed = ref_mv ? &sd : nullptr;
  job->subpel = subpel;
  job->angular = angular;
  job->cx = ctu_x * kCtu, job->cy = ctu_y * kCtu;
  for (int d = 0; d < 4; ++d)
    for (int ly = 0; ly < (1 << d); ++ly)
      for (int lx = 0; lx < (1 << d); ++lx) {
        int n = kCtu >> d, x0 = job->cx + lx * n, y0 = job->cy + ly * n;
        Node& nd = job->nodes[node_index(d, lx, ly)];
        nd = Node{};
        if (x0 >= c.w8 || y0 >= c.h8) nd.kind = 0;
        else if (x0 + n > c.w8 || y0 + n > c.h8) nd.kind = 1;
        else {
          nd.kind = 2;
          evaluate_leaf(c, r, x0, y0, n, R, job->s, job->seed, job->subpel, job->angular, &nd);
        }
        int64_t* o = rec + 14 * node_index(d, lx, ly);
        o[13] = nd.satd_angular_best;
        o[0] = nd.kind, o[1] = nd.mode, o[2] = nd.mx, o[3] = nd.my, o[4] = nd.sad;
        o[11] = nd.qmx, o[12] = nd.qmy;
        o[5] = nd.satd_inter, o[6] = nd.satd_planar, o[7] = nd.satd_dc, o[8] = nd.leaf_j;
        o[9] = nd.leaf_d, o[10] = nd.leaf_r;
      }
  delete job;
  return 0;
}

// Full coding-tree search of the listed CTUs (or all CTUs when ctu_list is
// null), threaded over CTUs.  Outputs (caller-allocated, host):
//   depth, mode: [h8/8][w8/8] u8; mv: [h8/8][w8/8][2] i16;
//   ctu_cost/dist/bits: [ceil(h/64)][ceil(w/64)] i64.
// bounds: null for full search, else [h8/8][w8/8][2] {lo, hi}.
// ref_mv: null for full search, else a seeded search (see make_seed).
// flags: bit 0 sub-pel refinement, bit 1 angular intra modes.
int orc_ctu_search(const uint8_t* cur, const uint8_t* ref, int w, int h, int stride, int qp,
                   int R, int flags, const uint8_t* bounds, const int16_t* ref_mv, int ref_w,
                   int ref_h, int refine_r, int seed_qpel, uint8_t* depth, uint8_t* mode,
                   int16_t* mv, int64_t* ctu_cost, int64_t* ctu_dist, int64_t* ctu_bits,
                   const int32_t* ctu_list, int n_list, int n_threads) {
  Seed sd{};
  if (!valid_pic(cur, w, h, stride) || !ref || R < 0 || R > 128 || qp < 0 || qp > 51 ||
      flags < 0 || flags > 3 || !depth || !mode || !mv || !ctu_cost || !ctu_dist ||
      !ctu_bits || !make_seed(ref_mv, ref_w, ref_h, refine_r, R, seed_qpel, &sd))
    return -1;
  const bool subpel = (flags & 1) != 0, angular = (flags & 2) != 0;
  const Seed* seed = ref_mv ? &sd : nullptr;
  Pic c = make_pic(cur, w, h, stride), r = make_pic(ref, w, h, stride);
  int ctw = (c.w8 + kCtu - 1) / kCtu, cth = (c.h8 + kCtu - 1) / kCtu;
  std::vector<int> list;
  if (ctu_list) {
    for (int i = 0; i < n_list; ++i) {
      if (ctu_list[i] < 0 || ctu_list[i] >= ctw * cth) return -1;
      list.push_back(ctu_list[i]);
    }
  } else {
    for (int i = 0; i < ctw * cth; ++i) list.push_back(i);
  }
  int64_t s = sqrt_lambda_q16(qp);
  std::atomic<int> next{0};
  auto worker = [&]() {
    CtuJob* job = new CtuJob();
    for (;;) {
      int k = next.fetch_add(1);
      if (k >= (int)list.size()) break;
      int t = list[k];
      *job = CtuJob{};
      job->cur = &c, job->ref = &r, job->R = R, job->s = s, job->bounds = bounds;
      job->seed = seed;
      job->subpel = subpel;
      job->angular = angular;
      job->cx = (t % ctw) * kCtu, job->cy = (t / ctw) * kCtu;
      bool leaf;
      Result root = best_tree(*job, 0, 0, 0, &leaf);
      write_tree(*job, 0, 0, 0, depth, mode, mv);
      ctu_cost[t] = root.j, ctu_dist[t] = root.d, ctu_bits[t] = root.r;
    }
    delete job;
  };
  if (n_threads <= 0) n_threads = (int)std::max(1u, std::thread::hardware_concurrency());
  n_threads = std::min<int>(n_threads, (int)list.size());
  std::vector<std::thread> pool;
  for (int i = 1; i < n_threads; ++i) pool.emplace_back(worker);
  worker();
  for (auto& th : pool) th.join();
  return 0;
}

// Depth bounds of a dependent representation from the reference depth map.
// Unit u at (8ux, 8uy): its centre maps to reference pixel
//   xr = min(((8ux + 4) * Wr) / Wd, Wr - 1), yr likewise with heights;
// d_r = ref_depth[yr / 8][xr / 8]; the scaled depth d_s is the smallest d in
// [0, 3] with (64 >> d) * Wr <= (64 >> d_r) * Wd (3 if none), and the bound is
// [max(0, d_s - delta_lo), min(3, d_s + delta_hi)].
int orc_depth_bounds(const uint8_t* ref_depth, int ref_w, int ref_h, int dep_w, int dep_h,
                     int delta_lo, int delta_hi, uint8_t* bounds_out) {
  if (!ref_depth || !bounds_out || ref_w <= 0 || ref_h <= 0 || dep_w <= 0 || dep_h <= 0 ||
      delta_lo < 0 || delta_hi < 0 || delta_lo > 3 || delta_hi > 3)
    return -1;
  int ruw = (ref_w + 7) / 8;
  int duw = (dep_w + 7) / 8, duh = (dep_h + 7) / 8;
  for (int uy = 0; uy < duh; ++uy)
    for (int ux = 0; ux < duw; ++ux) {
      int64_t xr = std::min<int64_t>(((int64_t)(8 * ux + 4) * ref_w) / dep_w, ref_w - 1);
      int64_t yr = std::min<int64_t>(((int64_t)(8 * uy + 4) * ref_h) / dep_h, ref_h - 1);
      int dr = ref_depth[(yr / 8) * ruw + xr / 8];
      int ds = 3;
      for (int d = 3; d >= 0; --d)
        if ((int64_t)(64 >> d) * ref_w <= (int64_t)(64 >> dr) * dep_w) ds = d;
      int64_t u = (int64_t)uy * duw + ux;
      bounds_out[2 * u] = (uint8_t)std::max(0, ds - delta_lo);
      bounds_out[2 * u + 1] = (uint8_t)std::min(3, ds + delta_hi);
    }
  return 0;
}

}  // extern "C"
