// Internal layouts shared by the host runtime and the HIP kernels of libmr.
#pragma once
#include <stdint.h>

namespace mr {

constexpr int kCtu = 64;
constexpr int kNodes = 85;          // 1 + 4 + 16 + 64 quad-tree nodes per CTU
constexpr int kMaxBands = 8;        // dy bands a CTU's search window may be split into
constexpr int kWaveSteps = 64;      // search tasks per wavefront step (one per lane)
constexpr int kRankBits = 11;       // rank field of the 32-bit arg-min key
constexpr uint32_t kCinv = 1050000u;  // cost field of candidates outside the window
constexpr uint64_t kKeyNone = ~0ull;
constexpr int kMaxStrip = 4;        // CTUs (wavefronts) per search workgroup
constexpr int kCurRingBytes = 512;  // per wavefront: two 16x16 regions of the current CTU
constexpr int kSplitWaves = 4;      // wavefronts of a split search item (one per quadrant)

// LDS dwords of the 64x64 SAD exchange of a split search item: two buffers
// (alternate steps) of three wavefronts x 64 lanes x 4D candidate sums.
__host__ __device__ constexpr int xch_dwords(int D) { return 2 * 3 * 64 * 4 * D; }

// Column margin of the padded reference of a seeded job with range R: the
// refinement loads reach 3 bytes left of -R and 20 bytes right of w8 - 8 + R.
__host__ __device__ inline int refine_pad_x(int R) { return (R + 24 + 3) & ~3; }
// Row margin: the refinement reaches R rows, the sub-pel patches R + 4.
__host__ __device__ inline int refine_pad_y(int R) { return R + 8; }

// Refinement key tables of a seeded job, built by the pad kernel in the job's
// scratch.  With c(v) = s * se(4 v) (the MV-bit term of one component, < 2^28)
// and i = v + R in [0, 2R]:
//   rk[i] = (c(dx) >> 16) * 2^9 + rank(i), rank ordering the 2R + 1 columns by
//           (c(dx) & 0xFFFF, i) over the whole range;
//   rd[rank(i)] = (c(dx) & 0xFFFF) * 2^17 + i;
//   ru[i] = c(dy) * 2^17 + i * (2R + 1).
// Within one window row, (SAD + (c >> 16)) * 2^9 + rank orders the candidates
// as their 64-bit keys do, and the row minimum m decodes to the key
// (m >> 9) * 2^33 + rd[m & 511] + ru[dy + R].
// Largest batch head (descriptors, items, lists) uploaded as a kernel's
// argument rather than by a copy from host memory.
constexpr size_t kUploadMaxBytes = 3584;

constexpr int kRtabSpan = 257;  // 2R + 1 for R <= 128
constexpr int kRankBitsR = 9;
constexpr size_t kRtabRk = 0;
constexpr size_t kRtabRd = 1056;                   // after rk, 8-byte aligned
constexpr size_t kRtabRu = kRtabRd + 8 * kRtabSpan;
constexpr size_t kRtabBytes = kRtabRu + 8 * kRtabSpan;

// Search work queues, one per XCD: queue q holds items [off[q], off[q + 1]).
// Their head counters are 256 bytes apart (kCounterStride words), so that
// atomics on different queues do not meet on one memory line.
constexpr int kQueues = 8;
constexpr int kCounterStride = 64;
constexpr size_t kCounterBytes = (size_t)kQueues * kCounterStride * 4;
struct QueueOffsets {
  int32_t off[kQueues + 1];
};

// One dependent's depth-bound computation (a batch of them is one launch).
struct BoundsJob {
  const uint8_t* ref_depth;  // device [ceil(ref_h / 8)][ceil(ref_w / 8)] depths
  uint8_t* out;              // device [ceil(dep_h / 8)][ceil(dep_w / 8)][2] {lo, hi}
  int ref_w, ref_h, dep_w, dep_h, dlo, dhi;
};
constexpr int kMaxBoundsJobs = 16;

// Search work item of a batch: x = job, y = row << 16 | first CTU column << 4 | band.
__host__ __device__ inline uint32_t pack_item_y(int row, int col0, int band) {
  return ((uint32_t)row << 16) | ((uint32_t)col0 << 4) | (uint32_t)band;
}

// Node index: depth offsets 0, 1, 5, 21, raster order inside a depth.
__host__ __device__ inline int node_index(int d, int lx, int ly) {
  return (d == 0 ? 0 : d == 1 ? 1 : d == 2 ? 5 : 21) + ly * (1 << d) + lx;
}

// Per-job search layout.  The (2R+1)^2 window is covered by tasks of
// 4 horizontal shifts (a quad) x D vertical shifts (a group), numbered group by
// group (task t: group t / Q, quad t % Q); tasks are dealt to wavefront steps of
// 64 in that order, and runs of whole steps form the dy bands.  When the task
// count is one more than a multiple of 64 and the last task holds a single
// candidate -- (dx, dy) = (R, R) -- that task is left out (one step less per
// CTU) and the prep kernel seeds every CU's key with that candidate instead.
struct SearchLayout {
  int32_t R, D, Q, G;           // range, group height, quads, groups
  int32_t ntasks, corner;       // tasks searched; 1: the (R, R) task is left out
  int32_t nbands, total_steps;
  int32_t band_g0[kMaxBands + 1];    // group of each band's first task
  int32_t band_step0[kMaxBands + 1]; // first global step of each band (+ end)
  int32_t win_rows_max, win_dwords;  // LDS window rows (largest band), dwords per row
};

// One frame pair's search job as seen by the kernels (stored in device memory;
// a batch is an array of these).
struct JobDesc {
  const uint8_t* cur;      // device luma
  const uint8_t* ref;
  int32_t w, h, stride;
  int32_t w8, h8, ctus_w, ctus_h;
  int32_t R, D, Q, nbands;
  int32_t ntasks;          // search tasks per CTU (see SearchLayout)
  int32_t corner;          // 1: keys start at the (R, R) candidate's (prep kernel)
  int32_t win_dwords;      // LDS window row length in dwords: Q + 16 * strip
  int32_t strip;           // CTUs per search workgroup (one wavefront each); 1 if split
  int32_t split;           // 1: a search item is one CTU whose quadrants go to the
                           // workgroup's four wavefronts
  int32_t ctu_start;       // first flattened CTU index of this job in its batch
  int32_t band_g0[kMaxBands + 1];
  int32_t band_step0[kMaxBands + 1];
  int64_t s;               // sqrt(lambda) in Q16
  const uint32_t* curpack; // [ctus][64 blocks][16 dwords]
  int32_t pack_cur;        // 1: the prep kernel packs curpack; 0: another job of the
                           // batch with the same current frame does (shared copy)
  int32_t pad_rows;        // 1: the pad kernel copies refpad's rows; 0: shared copy
  int32_t pad_row_start;   // first of this job's rows among the pad kernel's row blocks
                           // (the padding jobs' rows in job-list order; a job that pads
                           // nothing has the next padding job's start)
  uint64_t* keys;          // [ctus][85] arg-min keys J_me * 2^17 + candidate index
  const uint32_t* qtab;    // [steps][64 lanes][4D]
  const uint64_t* dtab;    // [steps][2048]
  const uint8_t* bounds;   // [U][V][2] or null
  uint8_t* elig;           // [ctus][85] 1 = node may be a leaf (inside and allowed)
  uint32_t* eligbits;      // [ctus][4] the same as a bit mask (bit n of word n / 32)
  uint8_t* okbits;         // [ctus][85] bit 0: the node may split, bit 1: it may be a leaf
                           // (the bounds rule; written by the prep kernel)
  // Seeded search (reference MV reuse with a refinement window); seed_mv null
  // means full search.
  const int16_t* seed_mv;  // [ceil(seed_h/8)][ceil(seed_w/8)][2] reference MVs
  int32_t seed_w, seed_h;  // dimensions of the picture the MVs belong to
  int32_t seed_r;          // refinement half-width r
  int32_t seed_qpel;       // 1: seed_mv in quarter-pel units
  int32_t rctu_start;      // first CTU of this job among the seeded jobs' CTUs
  uint8_t* rtab;           // refinement key tables (kRtabBytes), seeded jobs only
  uint32_t* seedc;         // [ctus][85] search centre of each CU, seeded jobs only:
                           // (uint16) dx | dy << 16 (written by the prep kernel)
  int32_t angular;         // 1: the leaf also scores the 33 angular intra modes
  // Intra SATDs shared by jobs of a batch with the same current frame (none of
  // them angular): the first such job's leaf writes, per node of every CTU,
  // {planar SATD, DC SATD} of every node inside the picture to `intra`
  // ([ctus][85][2]; null when no other job shares them); the others' leaf
  // (a later launch) reads them from `intra_src` and computes the inter SATDs
  // only.
  uint32_t* intra;
  const uint32_t* intra_src;
  uint64_t intra_users;    // bit k: job k of the batch takes this job's intra SATDs (bit 63:
                           // job 63 or later does); the SATDs are computed for the nodes
                           // eligible in this job or in one of them
  int32_t lctu_start;      // with shared intra SATDs: first CTU of this job among the
                           // CTUs of its leaf launch (jobs taking them, or the others)
  // Sub-pel refinement: per node {quarter-pel MV (qx | qy << 16), SATD}.
  int32_t subpel;
  int32_t sctu_start;      // first CTU of this job among the sub-pel jobs' CTUs
  uint32_t* subres;        // [ctus][85][2]
  // Padded reference (seeded or sub-pel jobs): rows [-pad_y, h8 + pad_y),
  // columns [-pad_x, w8 + pad_x), coordinates clamped to the picture.
  int32_t pad_x, pad_y, pad_pitch;
  uint8_t* refpad;         // [h8 + 2 pad_y][pad_pitch]
  uint8_t* depth;          // outputs
  uint8_t* mode;
  int16_t* mv;
  int64_t* ctu_cost;
  int64_t* ctu_dist;
  int64_t* ctu_bits;
};

}  // namespace mr
