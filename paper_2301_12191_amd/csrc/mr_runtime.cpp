// Host runtime of libmr: argument checks, search layouts, rank-ordered key
// tables, stream-ordered scratch and the C ABI entry points for one frame pair.
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

static constexpr size_t kLdsBudget = 64 * 1024;  // two search workgroups per CU

TileConfig default_tiles(int R, int n_ctus) {
  TileConfig tc;
  tc.D = R < 20 ? 2 : (R < 48 ? 4 : 8);
  const int span = 2 * R + 1, Q = (span + 3) / 4, G = (span + tc.D - 1) / tc.D;
  const size_t row_bytes = (size_t)(Q + 16) * 4;
  int nb = 1;
  while (nb < kMaxBands && nb < G) {
    const int B = (G + nb - 1) / nb;
    if ((size_t)(B * tc.D + 63) * row_bytes <= kLdsBudget) break;
    ++nb;
  }
  // Small jobs: split the window further so the grid has enough workgroups.
  while (nb < kMaxBands && (int64_t)n_ctus * nb < 1024 && (G + nb) / (nb + 1) >= 2) ++nb;
  tc.nbands = nb;
  return tc;
}

SearchLayout make_layout(int R, const TileConfig& tc) {
  SearchLayout L;
  std::memset(&L, 0, sizeof(L));
  const int span = 2 * R + 1;
  L.R = R;
  L.D = tc.D;
  L.Q = (span + 3) / 4;
  L.G = (span + tc.D - 1) / tc.D;
  L.nbands = std::max(1, std::min(std::min(tc.nbands, kMaxBands), L.G));
  L.band_step0[0] = 0;
  L.win_rows_max = 0;
  for (int b = 0; b <= L.nbands; ++b) L.band_g0[b] = (int)((int64_t)b * L.G / L.nbands);
  for (int b = 0; b < L.nbands; ++b) {
    const int B = L.band_g0[b + 1] - L.band_g0[b];
    const int tasks = B * L.Q;
    L.band_step0[b + 1] = L.band_step0[b] + (tasks + kWaveSteps - 1) / kWaveSteps;
    L.win_rows_max = std::max(L.win_rows_max, B * L.D + 63);
  }
  L.total_steps = L.band_step0[L.nbands];
  L.win_dwords = L.Q + 16;
  return L;
}

size_t search_lds_bytes(const SearchLayout& L) {
  return (size_t)L.win_rows_max * L.win_dwords * 4;
}

namespace {

struct TableKey {
  int device, qp, R, D, nbands;
  bool operator<(const TableKey& o) const {
    return std::tie(device, qp, R, D, nbands) < std::tie(o.device, o.qp, o.R, o.D, o.nbands);
  }
};

std::mutex g_tab_mu;
std::map<TableKey, KeyTables> g_tables;

struct Cand {
  uint32_t gamma, idx, C;
  int slot;  // lane * 4D + j * 4 + k
};

void build_tables(int qp, const SearchLayout& L, std::vector<uint32_t>& q,
                  std::vector<uint64_t>& dt) {
  const int R = L.R, D = L.D, span = 2 * R + 1, per_lane = 4 * D;
  const int64_t s = sqrt_lambda_q16(qp);
  q.assign((size_t)L.total_steps * kWaveSteps * per_lane, 0);
  dt.assign((size_t)L.total_steps * 2048, 0);
  std::vector<Cand> valid;
  std::vector<int> invalid;
  for (int b = 0; b < L.nbands; ++b) {
    const int g0 = L.band_g0[b], ntasks = (L.band_g0[b + 1] - g0) * L.Q;
    for (int st = 0; st < L.band_step0[b + 1] - L.band_step0[b]; ++st) {
      const int gstep = L.band_step0[b] + st;
      valid.clear();
      invalid.clear();
      for (int lane = 0; lane < kWaveSteps; ++lane) {
        const int task = st * kWaveSteps + lane;
        for (int j = 0; j < D; ++j)
          for (int k = 0; k < 4; ++k) {
            const int slot = lane * per_lane + j * 4 + k;
            bool ok = task < ntasks;
            int dx = 0, dy = 0;
            if (ok) {
              const int g = task / L.Q, qd = task % L.Q;
              dy = -R + (g0 + g) * D + j;
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
  const TableKey key{dev, qp, L.R, L.D, L.nbands};
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

static size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t job_scratch_bytes(int n_ctus) {
  return up256((size_t)n_ctus * 4096) + up256((size_t)n_ctus * kNodes * 8) +
         up256((size_t)n_ctus * kNodes);
}

void fill_job(JobDesc* jb, const mr_frame* cur, const mr_frame* ref, const mr_search_params* p,
              const uint8_t* bounds, const mr_search_out* out, const SearchLayout& L,
              const KeyTables& kt, void* scratch) {
  std::memset(jb, 0, sizeof(*jb));
  jb->cur = cur->luma;
  jb->ref = ref->luma;
  jb->w = cur->width;
  jb->h = cur->height;
  jb->stride = cur->stride;
  jb->w8 = (cur->width + 7) / 8 * 8;
  jb->h8 = (cur->height + 7) / 8 * 8;
  jb->ctus_w = (jb->w8 + kCtu - 1) / kCtu;
  jb->ctus_h = (jb->h8 + kCtu - 1) / kCtu;
  jb->R = L.R;
  jb->D = L.D;
  jb->Q = L.Q;
  jb->nbands = L.nbands;
  jb->win_dwords = L.win_dwords;
  for (int b = 0; b <= kMaxBands; ++b) {
    jb->band_g0[b] = L.band_g0[b];
    jb->band_step0[b] = L.band_step0[b];
  }
  jb->s = sqrt_lambda_q16(p->qp);
  const int n_ctus = jb->ctus_w * jb->ctus_h;
  uint8_t* sp = (uint8_t*)scratch;
  jb->curpack = (const uint32_t*)sp;
  sp += up256((size_t)n_ctus * 4096);
  jb->keys = (uint64_t*)sp;
  sp += up256((size_t)n_ctus * kNodes * 8);
  jb->elig = sp;
  jb->qtab = kt.qtab;
  jb->dtab = kt.dtab;
  jb->bounds = bounds;
  jb->depth = out->depth;
  jb->mode = out->mode;
  jb->mv = out->mv;
  jb->ctu_cost = out->ctu_cost;
  jb->ctu_dist = out->ctu_dist;
  jb->ctu_bits = out->ctu_bits;
}

static bool frame_ok(const mr_frame* f) {
  return f && f->luma && f->width >= 1 && f->height >= 1 && f->width <= 8192 &&
         f->height <= 8192 && f->stride >= f->width;
}

int validate_search(const mr_frame* cur, const mr_frame* ref, const mr_search_params* p,
                    const mr_search_out* out) {
  if (!frame_ok(cur) || !frame_ok(ref) || !p || !out) return MR_EINVAL;
  if (cur->width != ref->width || cur->height != ref->height || cur->stride != ref->stride)
    return MR_EINVAL;
  if (p->qp < 0 || p->qp > 51 || p->search_range < 0 || p->search_range > 128) return MR_EINVAL;
  if (!out->depth || !out->mode || !out->mv || !out->ctu_cost || !out->ctu_dist ||
      !out->ctu_bits)
    return MR_EINVAL;
  return MR_OK;
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
    default: return "unknown mr_status";
  }
}

int mr_ctu_search(const mr_frame* cur, const mr_frame* ref, const mr_search_params* p,
                  const uint8_t* bounds, mr_search_out* out, void* hip_stream) {
  int rc = validate_search(cur, ref, p, out);
  if (rc != MR_OK) return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  const int w8 = (cur->width + 7) / 8 * 8, h8 = (cur->height + 7) / 8 * 8;
  const int n_ctus = ((w8 + 63) / 64) * ((h8 + 63) / 64);
  const SearchLayout L = make_layout(p->search_range, default_tiles(p->search_range, n_ctus));
  KeyTables kt;
  rc = get_key_tables(p->qp, L, &kt);
  if (rc != MR_OK) return rc;
  void* scratch = nullptr;
  if (hipMallocAsync(&scratch, job_scratch_bytes(n_ctus), st) != hipSuccess) return MR_ENOMEM;
  JobDesc jb;
  fill_job(&jb, cur, ref, p, bounds, out, L, kt, scratch);
  hipError_t e = launch_prep1(jb, st);
  if (e == hipSuccess) e = launch_search1(jb, search_lds_bytes(L), st);
  if (e == hipSuccess) e = launch_leaf1(jb, st);
  const hipError_t ef = hipFreeAsync(scratch, st);
  if (e != hipSuccess || ef != hipSuccess) return MR_EHIP;
  return MR_OK;
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
