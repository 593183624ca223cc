// Host runtime of libmr: argument checks, search layouts, rank-ordered key
// tables, batch plans, and the single-pair C ABI entry points.
#include "mr_runtime.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>

namespace mr {

int64_t sqrt_lambda_q16(int qp) {
  const double lambda = 0.57 * std::exp2((qp - 12) / 3.0);
  return (int64_t)std::llround(std::sqrt(lambda) * 65536.0);
}

int se_bits(int v) {
  const uint32_t k = v > 0 ? 2u * (uint32_t)v - 1u : 2u * (uint32_t)(-(int64_t)v);
  return 2 * (31 - __builtin_clz(k + 1u)) + 1;
}

// ------------------------------------------------------------------------ tiles
namespace {
std::mutex g_tile_mu;
TileConfig g_tile_override[129];  // D == 0: none
}  // namespace

int set_tile_override(int R, const TileConfig& tc) {
  if (R < 0 || R > 128 ||
      !(tc.D == 0 || tc.D == 2 || tc.D == 4 || tc.D == 5 || tc.D == 6 || tc.D == 8))
    return MR_EINVAL;
  if (tc.D != 0 && (tc.nbands < 0 || tc.nbands > kMaxBands || tc.strip < 0 ||
                    tc.strip > kMaxStrip))
    return MR_EINVAL;
  if (tc.split < 0 || tc.split > 2) return MR_EINVAL;
  std::lock_guard<std::mutex> lk(g_tile_mu);
  g_tile_override[R] = tc.D ? tc : TileConfig{0, 0, 0, 0};
  return MR_OK;
}

bool get_tile_override(int R, TileConfig* tc) {
  std::lock_guard<std::mutex> lk(g_tile_mu);
  if (!g_tile_override[R].D) return false;
  *tc = g_tile_override[R];
  return true;
}

// Vertical shifts per lane when nothing overrides them, by the batch's
// dominant range R and its CTU count: the D whose steps waste the fewest
// lanes on candidates outside the window, where its registers allow three
// wavefronts per SIMD; at R >= 96 D = 8 (two wavefronts per SIMD), whose rows
// serve twice as many vertical shifts.  A small single picture at R < 20 keeps
// D = 2: three steps per CTU give its few CTUs three times as many work items.
int default_D(int R, int64_t ctus) {
  if (R < 20) return ctus < 256 ? 2 : 5;
  if (R >= 40 && R <= 56) return 5;
  if (R >= 96) return 8;
  return 4;
}

SearchLayout make_layout(int R, int D, int nbands) {
  SearchLayout L;
  std::memset(&L, 0, sizeof(L));
  const int span = 2 * R + 1;
  L.R = R;
  L.D = D;
  L.Q = (span + 3) / 4;
  L.G = (span + D - 1) / D;
  L.ntasks = L.Q * L.G;
  // The last task is the one holding (R, R); it holds nothing else when 2R is a
  // multiple of 4 and of D.  Leaving it out saves a step when it is alone in it.
  if (R > 0 && (2 * R) % 4 == 0 && (2 * R) % D == 0 && L.ntasks % kWaveSteps == 1) {
    L.corner = 1;
    L.ntasks -= 1;
  }
  L.total_steps = (L.ntasks + kWaveSteps - 1) / kWaveSteps;
  L.nbands = std::max(1, std::min(std::min(nbands, kMaxBands), L.total_steps));
  for (int b = 0; b <= L.nbands; ++b)
    L.band_step0[b] = (int)((int64_t)b * L.total_steps / L.nbands);
  for (int b = 0; b < L.nbands; ++b) {
    const int t0 = L.band_step0[b] * kWaveSteps;
    const int t1 = std::min(L.band_step0[b + 1] * kWaveSteps, L.ntasks);
    L.band_g0[b] = t0 / L.Q;
    const int g_last = (t1 - 1) / L.Q;
    L.win_rows_max = std::max(L.win_rows_max, (g_last - L.band_g0[b] + 1) * D + 63);
  }
  L.band_g0[L.nbands] = L.G;
  L.win_dwords = L.Q;  // + 16 * strip, added per job
  return L;
}

// The window is column-major with an odd pitch of (rows | 1) dwords.
size_t window_bytes(const SearchLayout& L, int strip) {
  return (size_t)(L.win_rows_max | 1) * (L.Q + 16 * strip) * 4 + (size_t)kCurRingBytes * strip;
}

int choose_bands(int R, int D, int strip, int ctus_w, int ctus_h, size_t lds_budget,
                 int min_items, int min_steps_per_band) {
  const int S = make_layout(R, D, 1).total_steps;
  int nb = 1;
  while (nb < kMaxBands && nb < S && window_bytes(make_layout(R, D, nb), strip) > lds_budget) ++nb;
  const int64_t strips = (int64_t)((ctus_w + strip - 1) / strip) * ctus_h;
  while (min_items > 0 && nb < kMaxBands && strips * nb < min_items &&
         (S + nb) / (nb + 1) >= min_steps_per_band)
    ++nb;
  return nb;
}

bool default_split(int R) { return R <= 64; }

// LDS budget per search workgroup: three workgroups per CU (the window plus
// a 512-byte current-CTU ring per wavefront).
static constexpr size_t kLdsBudget = 51 * 1024;

// ----------------------------------------------------------------------- tables
namespace {

struct TableKey {  // the tables follow the global steps, whatever the band split
  int device, qp, R, D;
  bool operator<(const TableKey& o) const {
    return std::tie(device, qp, R, D) < std::tie(o.device, o.qp, o.R, o.D);
  }
};

std::mutex g_tab_mu;
std::map<TableKey, KeyTables> g_tables;

struct Cand {
  uint32_t gamma, idx, C;
  int slot;  // lane * 4D + j * 4 + k
};

// For every wavefront step: each lane's 4D candidates get the constant
// q = C * 2048 + rank, C = (MV cost) >> 16, rank = position of the candidate
// among the step's valid candidates sorted by (MV cost & 0xFFFF, raster index).
// Then (SAD + C) * 2048 + rank orders the step's candidates exactly as
// (SAD * 65536 + MV cost, raster index).  dtab[rank] = (cost & 0xFFFF) << 17 | index.
void build_tables(int qp, const SearchLayout& L, std::vector<uint32_t>& q,
                  std::vector<uint64_t>& dt) {
  const int R = L.R, D = L.D, span = 2 * R + 1, per_lane = 4 * D;
  const int64_t s = sqrt_lambda_q16(qp);
  q.assign((size_t)L.total_steps * kWaveSteps * per_lane, 0);
  dt.assign((size_t)L.total_steps * 2048, 0);
  std::vector<Cand> valid;
  std::vector<int> invalid;
  {
    for (int gstep = 0; gstep < L.total_steps; ++gstep) {
      valid.clear();
      invalid.clear();
      for (int lane = 0; lane < kWaveSteps; ++lane) {
        const int task = gstep * kWaveSteps + lane;
        for (int j = 0; j < D; ++j)
          for (int k = 0; k < 4; ++k) {
            const int slot = lane * per_lane + j * 4 + k;
            bool ok = task < L.ntasks;
            int dx = 0, dy = 0;
            if (ok) {
              const int g = task / L.Q, qd = task % L.Q;
              dy = -R + g * D + j;
              dx = -R + 4 * qd + k;
              ok = dy <= R && dx <= R;
            }
            if (!ok) {
              invalid.push_back(slot);
              continue;
            }
            const int64_t c = s * (se_bits(4 * dx) + se_bits(4 * dy));
            valid.push_back(Cand{(uint32_t)(c & 0xFFFF), (uint32_t)((dy + R) * span + dx + R),
                                 (uint32_t)(c >> 16), slot});
          }
      }
      std::sort(valid.begin(), valid.end(), [](const Cand& a, const Cand& b) {
        return a.gamma != b.gamma ? a.gamma < b.gamma : a.idx < b.idx;
      });
      uint32_t* qs = q.data() + (size_t)gstep * kWaveSteps * per_lane;
      uint64_t* ds = dt.data() + (size_t)gstep * 2048;
      uint32_t rank = 0;
      for (const Cand& c : valid) {
        qs[c.slot] = c.C * 2048u + rank;
        ds[rank] = ((uint64_t)c.gamma << 17) | c.idx;
        ++rank;
      }
      for (int slot : invalid) qs[slot] = kCinv * 2048u + rank++;
    }
  }
}

}  // namespace

int get_key_tables(int qp, const SearchLayout& L, KeyTables* out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MR_EHIP;
  const TableKey key{dev, qp, L.R, L.D};
  std::lock_guard<std::mutex> lk(g_tab_mu);
  auto it = g_tables.find(key);
  if (it != g_tables.end()) {
    *out = it->second;
    return MR_OK;
  }
  std::vector<uint32_t> q;
  std::vector<uint64_t> dt;
  build_tables(qp, L, q, dt);
  void *dq = nullptr, *dd = nullptr;
  if (hipMalloc(&dq, q.size() * 4) != hipSuccess) return MR_ENOMEM;
  if (hipMalloc(&dd, dt.size() * 8) != hipSuccess) {
    (void)hipFree(dq);
    return MR_ENOMEM;
  }
  if (hipMemcpy(dq, q.data(), q.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dd, dt.data(), dt.size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(dq);
    (void)hipFree(dd);
    return MR_EHIP;
  }
  KeyTables kt{(const uint32_t*)dq, (const uint64_t*)dd};
  g_tables[key] = kt;
  *out = kt;
  return MR_OK;
}

// ------------------------------------------------------------------------ plans
static size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

static bool frame_ok(const mr_frame* f) {
  // The kernels address samples with 32-bit offsets.
  return f && f->luma && f->width >= 1 && f->height >= 1 && f->width <= 8192 &&
         f->height <= 8192 && f->stride >= f->width &&
         (int64_t)f->stride * (f->height - 1) + f->width <= (int64_t)INT32_MAX;
}

int validate_job(const mr_frame* cur, const mr_frame* ref, const mr_search_params* p,
                 const mr_search_out* out) {
  if (!frame_ok(cur) || !frame_ok(ref) || !p || !out) return MR_EINVAL;
  if (cur->width != ref->width || cur->height != ref->height || cur->stride != ref->stride)
    return MR_EINVAL;
  if (p->qp < 0 || p->qp > 51 || p->search_range < 0 || p->search_range > 128 || p->subpel < 0 ||
      p->subpel > 1 || p->angular < 0 || p->angular > 1)
    return MR_EINVAL;
  if (!out->depth || !out->mode || !out->mv || !out->ctu_cost || !out->ctu_dist ||
      !out->ctu_bits)
    return MR_EINVAL;
  return MR_OK;
}

int validate_seed(const mr_mv_seed* seed, const mr_search_params* p) {
  if (!seed) return MR_OK;
  if (!seed->ref_mv || seed->ref_w < 1 || seed->ref_h < 1 || seed->ref_w > 8192 ||
      seed->ref_h > 8192 || seed->refine_range < 0 || seed->refine_range > p->search_range ||
      seed->quarter_pel < 0 || seed->quarter_pel > 1)
    return MR_EINVAL;
  return MR_OK;
}

void set_job_seed(JobDesc& jb, const mr_mv_seed* seed) {
  jb.seed_mv = seed ? seed->ref_mv : nullptr;
  jb.seed_w = seed ? seed->ref_w : 0;
  jb.seed_h = seed ? seed->ref_h : 0;
  jb.seed_r = seed ? seed->refine_range : 0;
  jb.seed_qpel = seed ? seed->quarter_pel : 0;
}

int device_cu_count() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (!cached[dev]) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n <= 0)
      n = 256;
    cached[dev] = n;
  }
  return cached[dev];
}

size_t device_lds_max() {
  static size_t cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 64 * 1024;
  if (!cached[dev]) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        n <= 0)
      n = 64 * 1024;
    cached[dev] = (size_t)n;
  }
  return cached[dev];
}

// A frame's identity for sharing work between jobs of a batch: its memory and
// geometry (plus, for padded references, the margins).
using FrameKey = std::tuple<const uint8_t*, int, int, int, int, int>;
static FrameKey frame_key(const mr_frame* f, int mx = 0, int my = 0) {
  return FrameKey{f->luma, f->width, f->height, f->stride, mx, my};
}

int make_plan(const mr_frame* const* cur, const mr_frame* const* ref,
              const mr_search_params* const* p, const uint8_t* const* bounds,
              const mr_search_out* const* out, const mr_mv_seed* const* seeds, int n_jobs,
              bool materialize_items, Plan* P) {
  if (n_jobs < 1 || n_jobs > (1 << 20)) return MR_EINVAL;
  auto seed_of = [&](int j) { return seeds ? seeds[j] : nullptr; };
  for (int j = 0; j < n_jobs; ++j) {
    int rc = validate_job(cur[j], ref[j], p[j], out[j]);
    if (rc == MR_OK) rc = validate_seed(seed_of(j), p[j]);
    if (rc != MR_OK) return rc;
  }
  // Batch-wide D and strip from the full-search job with the most search work.
  int heavy = 0;
  double heavy_work = -1;
  int max_ctus_w = 1;
  for (int j = 0; j < n_jobs; ++j) {
    if (seed_of(j)) continue;
    const double r = 2.0 * p[j]->search_range + 1;
    const double work = r * r * (double)cur[j]->width * cur[j]->height;
    if (work > heavy_work) heavy_work = work, heavy = j;
    max_ctus_w = std::max(max_ctus_w, ((cur[j]->width + 7) / 8 * 8 + 63) / 64);
  }
  TileConfig tc{0, 0, 0, 0};
  const bool ov = get_tile_override(p[heavy]->search_range, &tc);
  int64_t fs_ctus = 0;  // CTUs of the full-search jobs
  for (int j = 0; j < n_jobs; ++j)
    if (!seed_of(j))
      fs_ctus += (int64_t)(((cur[j]->width + 7) / 8 * 8 + 63) / 64) *
                 (((cur[j]->height + 7) / 8 * 8 + 63) / 64);
  P->D = ov ? tc.D : default_D(p[heavy]->search_range, fs_ctus);
  P->strip = (ov && tc.strip) ? tc.strip : std::min(kMaxStrip, max_ctus_w);
  // Split jobs need a workgroup of four wavefronts; a batch with some keeps
  // strips of four for its other jobs.
  auto split_of = [&](int R) {
    TileConfig t;
    const int sp = get_tile_override(R, &t) ? t.split : 0;
    return sp == 2 || (sp == 0 && default_split(R));
  };
  bool any_split = false;
  for (int j = 0; j < n_jobs; ++j)
    if (!seed_of(j) && split_of(p[j]->search_range)) any_split = true;
  if (any_split) P->strip = kMaxStrip;
  P->n_jobs = n_jobs;
  P->jobs.assign(n_jobs, JobDesc{});
  P->job_off.assign(n_jobs, 0);
  P->cur_owner.assign(n_jobs, -1);
  P->pad_owner.assign(n_jobs, -1);
  // Jobs with the same current frame and no angular modes share the first
  // one's planar and DC SATDs (QP-independent); that one writes them for all.
  P->intra_owner.assign(n_jobs, -1);
  P->intra_owned.assign(n_jobs, 0);
  P->any_shared_intra = false;
  std::map<FrameKey, int> first_cur, first_intra, first_pad;
  for (int j = 0; j < n_jobs; ++j) {
    if (p[j]->angular) continue;
    auto ins = first_intra.emplace(frame_key(cur[j]), j);
    if (!ins.second) {
      P->intra_owner[j] = ins.first->second;
      P->intra_owned[ins.first->second] = 1;
      P->any_shared_intra = true;
    }
  }
  P->items.clear();
  P->rlist.clear();
  P->slist.clear();
  P->plist.clear();
  P->n_rjobs = P->n_rctus = P->max_r = 0;
  P->n_sjobs = P->n_sctus = 0;
  P->pad_rows_total = 0;
  P->any_angular = false;
  P->n_ctus = 0;
  P->scratch_bytes = 0;
  P->lds_bytes = 0;
  int64_t total_items = 0;
  const int min_items = n_jobs == 1 ? 3 * device_cu_count() : 0;
  struct Work {
    int64_t cost;
    uint32_t job, y;
  };
  // Per job, its items strip by strip (a strip's bands consecutive) and the
  // strip's band count.
  std::vector<std::vector<Work>> jwork(materialize_items ? n_jobs : 0);
  std::vector<int> jnb(n_jobs, 1);
  for (int j = 0; j < n_jobs; ++j) {
    JobDesc& jb = P->jobs[j];
    std::memset(&jb, 0, sizeof(jb));
    const int R = p[j]->search_range;
    jb.cur = cur[j]->luma;
    jb.ref = ref[j]->luma;
    jb.w = cur[j]->width;
    jb.h = cur[j]->height;
    jb.stride = cur[j]->stride;
    jb.w8 = (jb.w + 7) / 8 * 8;
    jb.h8 = (jb.h + 7) / 8 * 8;
    jb.ctus_w = (jb.w8 + kCtu - 1) / kCtu;
    jb.ctus_h = (jb.h8 + kCtu - 1) / kCtu;
    const int n_ctus = jb.ctus_w * jb.ctus_h;
    jb.R = R;
    jb.ctu_start = P->n_ctus;
    jb.s = sqrt_lambda_q16(p[j]->qp);
    jb.bounds = bounds[j];
    jb.depth = out[j]->depth;
    jb.mode = out[j]->mode;
    jb.mv = out[j]->mv;
    jb.ctu_cost = out[j]->ctu_cost;
    jb.ctu_dist = out[j]->ctu_dist;
    jb.ctu_bits = out[j]->ctu_bits;
    P->job_off[j] = P->scratch_bytes;
    // Jobs that read the same current frame (e.g. one pair at several QPs)
    // share one packed copy of its CTUs.
    {
      auto ins = first_cur.emplace(frame_key(cur[j]), j);
      P->cur_owner[j] = ins.second ? -1 : ins.first->second;
    }
    jb.pack_cur = P->cur_owner[j] < 0 ? 1 : 0;
    P->scratch_bytes += (jb.pack_cur ? up256((size_t)n_ctus * 4096) : 0) +
                        up256((size_t)n_ctus * kNodes * 8) + 2 * up256((size_t)n_ctus * kNodes) +
                        up256((size_t)n_ctus * 16) +
                        (P->intra_owned[j] ? up256((size_t)n_ctus * kNodes * 8) : 0);
    P->n_ctus += n_ctus;
    jb.subpel = p[j]->subpel;
    jb.angular = p[j]->angular;
    if (jb.angular) P->any_angular = true;
    if (jb.subpel) {
      jb.sctu_start = P->n_sctus;
      P->scratch_bytes += up256((size_t)n_ctus * kNodes * 8);  // subres
      P->slist.push_back(j);
      P->n_sjobs += 1;
      P->n_sctus += n_ctus;
    }
    P->pad_owner[j] = -1;
    if (seed_of(j) || jb.subpel) {
      jb.pad_x = refine_pad_x(R);
      jb.pad_y = refine_pad_y(R);
      jb.pad_pitch = jb.w8 + 2 * jb.pad_x;
      // The same reference frame with the same margins (same R): one copy.
      auto ins = first_pad.emplace(frame_key(ref[j], jb.pad_x, jb.pad_y), j);
      P->pad_owner[j] = ins.second ? -1 : ins.first->second;
      jb.pad_rows = P->pad_owner[j] < 0 ? 1 : 0;
      const int64_t pad_bytes = (int64_t)(jb.h8 + 2 * jb.pad_y) * jb.pad_pitch;
      if (jb.pad_rows) P->scratch_bytes += up256((size_t)pad_bytes);
      jb.pad_row_start = P->pad_rows_total;
      if (jb.pad_rows) P->pad_rows_total += jb.h8 + 2 * jb.pad_y;
      P->plist.push_back(j);
    }
    if (seed_of(j)) {
      // Seeded: refinement around reference MVs instead of the full search.
      set_job_seed(jb, seed_of(j));
      P->scratch_bytes += up256(kRtabBytes) + up256((size_t)n_ctus * kNodes * 4);  // + seedc
      jb.rctu_start = P->n_rctus;
      P->rlist.push_back(j);
      P->n_rjobs += 1;
      P->n_rctus += n_ctus;
      P->max_r = std::max(P->max_r, jb.seed_r);
      continue;
    }
    // A split job is searched one CTU per workgroup (window of one CTU) and
    // its bands may be single steps: each item is a quarter CTU per wavefront.
    const bool split = split_of(R);
    const size_t xch_bytes = split ? (size_t)xch_dwords(P->D) * 4 : 0;
    const size_t ring_extra = split ? (size_t)kCurRingBytes * (kSplitWaves - 1) : 0;
    int nb = split ? choose_bands(R, P->D, 1, jb.ctus_w, jb.ctus_h,
                                  kLdsBudget - xch_bytes - ring_extra, min_items, 1)
                   : choose_bands(R, P->D, P->strip, jb.ctus_w, jb.ctus_h, kLdsBudget, min_items);
    TileConfig tj;
    if (get_tile_override(R, &tj) && tj.D == P->D && tj.nbands) nb = tj.nbands;
    const SearchLayout L = make_layout(R, P->D, nb);
    KeyTables kt{nullptr, nullptr};
    if (!P->defer_tables) {
      const int rc = get_key_tables(p[j]->qp, L, &kt);
      if (rc != MR_OK) return rc;
    }
    jb.D = P->D;
    jb.Q = L.Q;
    jb.ntasks = L.ntasks;
    jb.corner = L.corner;
    jb.nbands = L.nbands;
    jb.split = split ? 1 : 0;
    jb.strip = split ? 1 : P->strip;
    jb.win_dwords = L.Q + 16 * jb.strip;
    for (int b = 0; b <= kMaxBands; ++b) {
      jb.band_g0[b] = L.band_g0[b];
      jb.band_step0[b] = L.band_step0[b];
    }
    jb.qtab = kt.qtab;
    jb.dtab = kt.dtab;
    // LDS: the window (plus, split, the 64x64 exchange after it), then one
    // ring per wavefront of the launch.
    P->lds_bytes = std::max(P->lds_bytes, split ? window_bytes(L, 1) + xch_bytes + ring_extra
                                                : window_bytes(L, P->strip));
    const int spr = (jb.ctus_w + jb.strip - 1) / jb.strip;
    total_items += (int64_t)spr * jb.ctus_h * L.nbands;
    jnb[j] = L.nbands;
    if (materialize_items) {
      for (int row = 0; row < jb.ctus_h; ++row)
        for (int sidx = 0; sidx < spr; ++sidx)
          for (int b = 0; b < L.nbands; ++b) {
            const int steps = L.band_step0[b + 1] - L.band_step0[b];
            const int rows = (L.band_g0[b + 1] - L.band_g0[b]) * P->D + 63;
            // A partial strip spreads its CTUs' steps over all the strip's
            // wavefronts; a split item gives each wavefront a quarter CTU.
            const int sw = std::min(jb.strip, jb.ctus_w - sidx * jb.strip);
            const int64_t span = ((int64_t)sw * steps + jb.strip - 1) / jb.strip;
            const int64_t cost = span * (split ? 1024 : 4096) + rows;  // compute + staging
            jwork[j].push_back(Work{cost, (uint32_t)j, pack_item_y(row, sidx * jb.strip, b)});
          }
    }
  }
  // The two leaf launches of shared intra SATDs: jobs that take none, then the others.
  P->llist.clear();
  P->n_ljobs0 = P->n_lctus0 = P->n_lctus1 = 0;
  if (P->any_shared_intra) {
    for (int pass = 0; pass < 2; ++pass)
      for (int j = 0; j < n_jobs; ++j) {
        if ((P->intra_owner[j] >= 0) != (pass == 1)) continue;
        JobDesc& jb = P->jobs[j];
        int& cnt = pass == 0 ? P->n_lctus0 : P->n_lctus1;
        jb.lctu_start = cnt;
        cnt += jb.ctus_w * jb.ctus_h;
        P->llist.push_back(j);
        if (pass == 0) P->n_ljobs0 += 1;
      }
  }
  if (total_items > ((int64_t)1 << 30)) return MR_EINVAL;
  if (P->lds_bytes > device_lds_max()) return MR_EINVAL;  // a forced tile shape too large
  P->n_items = (int)total_items;
  // One queue per XCD: workgroups are dealt to the 8 XCDs round-robin, and a
  // workgroup starts on queue blockIdx.x mod 8, then takes from the others once
  // its own is empty.  Each job's strips, every strip with all its bands, are
  // cut into kQueues contiguous runs of equal cost, run q to queue q, so that
  // one XCD's L2 holds the current CTUs and window rows of a region of every
  // picture.  Each queue is in the order of one global queue: longest items
  // first (heavy search ranges and long bands start early, small ones fill the
  // tail).
  if (materialize_items) {
    std::vector<std::vector<Work>> qs(kQueues);
    for (int j = 0; j < n_jobs; ++j) {
      const std::vector<Work>& w = jwork[j];
      const size_t nb = (size_t)jnb[j];
      int64_t total = 0;
      for (const Work& x : w) total += x.cost;
      int64_t acc = 0;
      for (size_t u = 0; u < w.size(); u += nb) {  // one strip and its bands
        int64_t c = 0;
        for (size_t k = 0; k < nb; ++k) c += w[u + k].cost;
        const int q = total > 0 ? (int)std::min<int64_t>(kQueues - 1,
                                                         (acc + c / 2) * kQueues / total)
                                : 0;
        qs[q].insert(qs[q].end(), w.begin() + u, w.begin() + u + nb);
        acc += c;
      }
    }
    P->items.clear();
    P->items.reserve((size_t)total_items);
    P->qoff.off[0] = 0;
    for (int q = 0; q < kQueues; ++q) {
      std::stable_sort(qs[q].begin(), qs[q].end(),
                       [](const Work& a, const Work& b) { return a.cost > b.cost; });
      for (const Work& x : qs[q]) P->items.push_back(make_uint2(x.job, x.y));
      P->qoff.off[q + 1] = (int32_t)P->items.size();
    }
  } else {
    // One job, items implicit (index = strip * bands + band): runs of whole strips.
    const int64_t nb = jnb[0], strips = total_items / nb;
    for (int q = 0; q < kQueues; ++q) P->qoff.off[q] = (int32_t)(strips * q / kQueues * nb);
    P->qoff.off[kQueues] = (int32_t)total_items;
  }
  if (P->n_items > 0) {
    const int occ = std::max(1, search_occupancy(P->D, P->strip, P->lds_bytes));
    P->n_wg = (int)std::min<int64_t>(P->n_items, (int64_t)occ * device_cu_count());
  } else {
    P->n_wg = 0;
  }
  return MR_OK;
}

void bind_scratch(Plan& P, uint8_t* base) {
  for (int j = 0; j < P.n_jobs; ++j) {
    JobDesc& jb = P.jobs[j];
    const int n_ctus = jb.ctus_w * jb.ctus_h;
    uint8_t* sp = base + P.job_off[j];
    if (P.cur_owner[j] < 0) {
      jb.curpack = (const uint32_t*)sp;
      sp += up256((size_t)n_ctus * 4096);
    } else {
      jb.curpack = P.jobs[P.cur_owner[j]].curpack;  // owners come first
    }
    jb.keys = (uint64_t*)sp;
    sp += up256((size_t)n_ctus * kNodes * 8);
    jb.elig = sp;
    sp += up256((size_t)n_ctus * kNodes);
    jb.eligbits = (uint32_t*)sp;
    sp += up256((size_t)n_ctus * 16);
    jb.okbits = sp;
    sp += up256((size_t)n_ctus * kNodes);
    jb.intra = nullptr;
    jb.intra_src = nullptr;
    jb.intra_users = 0;  // owners come first: set below by the jobs that take theirs
    if (P.intra_owner[j] >= 0) {
      JobDesc& ow = P.jobs[P.intra_owner[j]];
      jb.intra_src = ow.intra;
      ow.intra_users |= 1ull << std::min(j, 63);
    } else if (P.intra_owned[j]) {
      jb.intra = (uint32_t*)sp;
      sp += up256((size_t)n_ctus * kNodes * 8);
    }
    jb.subres = nullptr;
    if (jb.subpel) {
      jb.subres = (uint32_t*)sp;
      sp += up256((size_t)n_ctus * kNodes * 8);
    }
    jb.rtab = nullptr;
    jb.seedc = nullptr;
    if (jb.seed_mv) {
      jb.rtab = sp;
      sp += up256(kRtabBytes);
      jb.seedc = (uint32_t*)sp;
      sp += up256((size_t)n_ctus * kNodes * 4);
    }
    jb.refpad = nullptr;
    if (jb.seed_mv || jb.subpel)
      jb.refpad = P.pad_owner[j] < 0 ? sp : P.jobs[P.pad_owner[j]].refpad;
  }
}

hipError_t launch_plan(const Plan& P, JobDesc* jobs_d, const uint2* items_d, const PlanLists& L,
                       uint32_t* counter, hipStream_t st, StageEvents* ev) {
  hipError_t e = launch_prep(jobs_d, P.n_jobs, P.n_ctus, counter, st);
  if (ev) profile_mark(ev, 1, st);
  if (e == hipSuccess && !P.plist.empty())
    e = launch_pad(jobs_d, L.plist, (int)P.plist.size(), P.pad_rows_total, st);
  if (e == hipSuccess && P.n_items > 0)
    e = launch_search(jobs_d, items_d, P.qoff, P.D, P.strip, P.n_wg, P.lds_bytes, counter, st);
  if (e == hipSuccess && P.n_rjobs > 0)
    e = launch_refine(jobs_d, L.rlist, P.n_rjobs, P.n_rctus, P.max_r, st);
  if (ev) profile_mark(ev, 2, st);
  if (e == hipSuccess && P.n_sjobs > 0)
    e = launch_subpel(jobs_d, L.slist, P.n_sjobs, P.n_sctus, st);
  if (ev) profile_mark(ev, 3, st);
  if (e == hipSuccess)
    e = launch_leaf(jobs_d, P.n_jobs, P.n_ctus, P.any_angular,
                    P.any_shared_intra ? L.llist : nullptr, P.n_ljobs0, P.n_lctus0, P.n_lctus1,
                    st);
  if (ev) profile_mark(ev, 4, st);
  return e;
}

// -------------------------------------------------------------------- profiling
namespace {
struct ProfileState {
  std::mutex mu;
  bool on = false;
  std::vector<StageEvents> pending;
  double ms[4] = {0, 0, 0, 0};
  int64_t n[4] = {0, 0, 0, 0};
};
ProfileState g_prof;
}  // namespace

bool profile_on() {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  return g_prof.on;
}

int profile_begin(StageEvents* ev, hipStream_t st) {
  for (auto& x : ev->e)
    if (hipEventCreate(&x) != hipSuccess) return MR_EHIP;
  return hipEventRecord(ev->e[0], st) == hipSuccess ? MR_OK : MR_EHIP;
}

void profile_mark(StageEvents* ev, int k, hipStream_t st) { (void)hipEventRecord(ev->e[k], st); }

void profile_push(const StageEvents& ev) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.pending.push_back(ev);
}

}  // namespace mr

using namespace mr;

extern "C" {

const char* mr_status_str(int status) {
  switch (status) {
    case MR_OK: return "MR_OK";
    case MR_EINVAL: return "MR_EINVAL: invalid argument";
    case MR_ENOMEM: return "MR_ENOMEM: allocation failed";
    case MR_EAGAIN: return "MR_EAGAIN: queue full or memory budget exhausted";
    case MR_EDEPEND: return "MR_EDEPEND: reference job missing";
    case MR_EHIP: return "MR_EHIP: HIP runtime error";
    case MR_ETIMEOUT: return "MR_ETIMEOUT: timed out";
    case MR_ESTATE: return "MR_ESTATE: invalid state for this call";
    case MR_ESCRATCH: return "MR_ESCRATCH: request exceeds the fixed scratch of the allocation-free search";
    default: return "unknown mr_status";
  }
}

int mr_ctu_search_seeded(const mr_frame* cur, const mr_frame* ref, const mr_search_params* p,
                         const uint8_t* bounds, const mr_mv_seed* seed, mr_search_out* out,
                         void* hip_stream) {
  hipStream_t st = (hipStream_t)hip_stream;
  Plan P;
  const mr_search_out* o = out;
  int rc = make_plan(&cur, &ref, &p, &bounds, &o, &seed, 1, false, &P);
  if (rc != MR_OK) return rc;
  // Scratch: job descriptor, queue counter, per-job buffers.
  const size_t head = up256(sizeof(JobDesc)) + kCounterBytes;
  uint8_t* scratch = nullptr;
  if (hipMallocAsync((void**)&scratch, head + P.scratch_bytes, st) != hipSuccess) return MR_ENOMEM;
  bind_scratch(P, scratch + head);
  JobDesc* jobs_d = (JobDesc*)scratch;
  uint32_t* counter = (uint32_t*)(scratch + up256(sizeof(JobDesc)));
  StageEvents ev{};
  const bool prof = profile_on() && profile_begin(&ev, st) == MR_OK;
  hipError_t e = launch_store_job(P.jobs[0], jobs_d, st);
  if (e == hipSuccess)
    e = launch_plan(P, jobs_d, nullptr, PlanLists{nullptr, nullptr, nullptr, nullptr}, counter, st,
                    prof ? &ev : nullptr);
  if (prof) profile_push(ev);
  const hipError_t ef = hipFreeAsync(scratch, st);
  if (e != hipSuccess || ef != hipSuccess) return MR_EHIP;
  return MR_OK;
}

int mr_ctu_search(const mr_frame* cur, const mr_frame* ref, const mr_search_params* p,
                  const uint8_t* bounds, mr_search_out* out, void* hip_stream) {
  return mr_ctu_search_seeded(cur, ref, p, bounds, nullptr, out, hip_stream);
}

int64_t mr_sqrt_lambda_q16(int32_t qp) { return qp < 0 || qp > 51 ? -1 : sqrt_lambda_q16(qp); }

int32_t mr_se_bits(int32_t v) {
  return (v > (1 << 29) || v < -(1 << 29)) ? -1 : se_bits(v);
}

int mr_set_tiles(int32_t search_range, int32_t d, int32_t nbands) {
  if (d != 0 && (nbands < 1 || nbands > kMaxBands)) return MR_EINVAL;
  return set_tile_override(search_range, TileConfig{d, nbands, 0, 0});
}

int mr_set_tiles3(int32_t search_range, int32_t d, int32_t nbands, int32_t strip) {
  if (d != 0 && (nbands < 1 || nbands > kMaxBands || strip < 0 || strip > kMaxStrip))
    return MR_EINVAL;
  return set_tile_override(search_range, TileConfig{d, nbands, strip, 0});
}

int mr_set_tiles4(int32_t search_range, int32_t d, int32_t nbands, int32_t strip,
                  int32_t split) {
  if (d != 0 && (nbands < 0 || nbands > kMaxBands || strip < 0 || strip > kMaxStrip ||
                 split < 0 || split > 2))
    return MR_EINVAL;
  return set_tile_override(search_range, TileConfig{d, nbands, strip, split});
}

int mr_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.on = on != 0;
  return MR_OK;
}

int mr_profile_read(mr_profile* out, int reset) {
  if (!out) return MR_EINVAL;
  std::lock_guard<std::mutex> lk(g_prof.mu);
  int rc = MR_OK;
  for (auto& ev : g_prof.pending) {
    if (hipEventSynchronize(ev.e[4]) != hipSuccess) rc = MR_EHIP;
    for (int k = 0; k < 4; ++k) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev.e[k], ev.e[k + 1]) != hipSuccess) rc = MR_EHIP;
      g_prof.ms[k] += ms;
      g_prof.n[k] += 1;
    }
    for (auto& x : ev.e) (void)hipEventDestroy(x);
  }
  g_prof.pending.clear();
  for (int k = 0; k < 4; ++k) {
    out->ms[k] = g_prof.ms[k];
    out->launches[k] = g_prof.n[k];
    if (reset) g_prof.ms[k] = 0, g_prof.n[k] = 0;
  }
  return rc;
}

int mr_depth_bounds(const uint8_t* ref_depth, int32_t ref_w, int32_t ref_h, int32_t dep_w,
                    int32_t dep_h, int32_t delta_lo, int32_t delta_hi, uint8_t* bounds_out,
                    void* hip_stream) {
  if (!ref_depth || !bounds_out || ref_w < 1 || ref_h < 1 || dep_w < 1 || dep_h < 1 ||
      ref_w > 8192 || ref_h > 8192 || dep_w > 8192 || dep_h > 8192 || delta_lo < 0 ||
      delta_lo > 3 || delta_hi < 0 || delta_hi > 3)
    return MR_EINVAL;
  if (launch_depth_bounds(ref_depth, ref_w, ref_h, dep_w, dep_h, delta_lo, delta_hi, bounds_out,
                          (hipStream_t)hip_stream) != hipSuccess)
    return MR_EHIP;
  return MR_OK;
}

}  // extern "C"
