// Allocation-free coding-tree search: mr_ctu_search_seeded's kernels over one
// fixed, file-scope device buffer instead of stream-ordered allocations.
//
// The buffer holds, in this order: the job descriptor, the search queue
// counters, the rank-ordered arg-min key tables of the job's (QP, R, D), and
// the per-job scratch of the plan (packed current CTUs, keys, eligibility,
// and for seeded / sub-pel jobs the padded reference and sub-pel results).
// The key tables are built on the device by key_table_kernel, so a call makes
// no host-to-device copy and no allocation of any kind on the device.
#include <hip/hip_runtime.h>

#include <mutex>

#include "mr_device.h"
#include "mr_runtime.h"

namespace mr {

constexpr size_t kNoAllocBytes = MR_NOALLOC_SCRATCH_BYTES;

// One copy per GPU, resident until the process ends.  Host code must not
// pass this name to a kernel: it uses the device address from
// hipGetSymbolAddress (noalloc_scratch below).
static __device__ __align__(256) uint8_t scratch[kNoAllocBytes];

namespace {

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

std::mutex g_scratch_mu;
uint8_t* g_scratch_ptr[64];  // device address of `scratch`, per device

// Device address of this device's scratch array, looked up once per device
// with that device current.
int noalloc_scratch(uint8_t** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return MR_EHIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MR_EHIP;
    g_scratch_ptr[dev] = (uint8_t*)p;
  }
  *out = g_scratch_ptr[dev];
  return MR_OK;
}

}  // namespace

// The key tables of one wavefront step (workgroup blockIdx.x), as the host
// builder of the cached tables defines them: slot lane * 4D + 4j + k holds
// candidate dx = -R + 4 (task % Q) + k, dy = -R + D (task / Q) + j of task
// step * 64 + lane, valid if the task exists and dx, dy <= R.  With
// c = s (se(4 dx) + se(4 dy)), a valid slot gets q = (c >> 16) * 2048 + rank,
// rank = its position among the step's valid slots ordered by
// (c & 0xFFFF, raster index), and dtab[rank] = (c & 0xFFFF) << 17 | raster
// index; invalid slots take the ranks after the valid ones in slot order with
// the cost field kCinv.  dtab entries past the valid ranks are zero.
__global__ __launch_bounds__(256) void key_table_kernel(int R, int D, int Q, int ntasks, int64_t s,
                                                        uint32_t* __restrict__ qtab,
                                                        uint64_t* __restrict__ dtab) {
  __shared__ uint64_t key[kWaveSteps * 4 * 8];  // (c & 0xFFFF) << 32 | index; ~0: invalid
  __shared__ uint32_t cfield[kWaveSteps * 4 * 8];
  __shared__ int s_nvalid;
  const int gstep = blockIdx.x, per_lane = 4 * D, nslots = kWaveSteps * per_lane;
  const int span = 2 * R + 1;
  if (threadIdx.x == 0) s_nvalid = 0;
  __syncthreads();
  int nv = 0;
  for (int slot = threadIdx.x; slot < nslots; slot += blockDim.x) {
    const int lane = slot / per_lane, j = (slot % per_lane) >> 2, k = slot & 3;
    const int task = gstep * kWaveSteps + lane;
    uint64_t kv = ~0ull;
    uint32_t C = kCinv;
    if (task < ntasks) {
      const int g = task / Q, qd = task % Q;
      const int dy = -R + g * D + j, dx = -R + 4 * qd + k;
      if (dy <= R && dx <= R) {
        const int64_t c = s * (int64_t)(se_bits_dev(4 * dx) + se_bits_dev(4 * dy));
        kv = ((uint64_t)(c & 0xFFFF) << 32) | (uint64_t)((dy + R) * span + dx + R);
        C = (uint32_t)(c >> 16);
        ++nv;
      }
    }
    key[slot] = kv;
    cfield[slot] = C;
  }
  atomicAdd(&s_nvalid, nv);
  __syncthreads();
  const int nvalid = s_nvalid;
  uint32_t* qs = qtab + (size_t)gstep * nslots;
  uint64_t* ds = dtab + (size_t)gstep * 2048;
  for (int slot = threadIdx.x; slot < nslots; slot += blockDim.x) {
    const uint64_t me = key[slot];
    uint32_t rank = 0;
    if (me != ~0ull) {
      for (int t = 0; t < nslots; ++t) rank += key[t] < me ? 1u : 0u;  // invalid keys are larger
      ds[rank] = ((me >> 32) << 17) | (me & 0xFFFFFFFFull);
    } else {
      rank = (uint32_t)nvalid;
      for (int t = 0; t < slot; ++t) rank += key[t] == ~0ull ? 1u : 0u;
    }
    qs[slot] = cfield[slot] * 2048u + rank;
  }
  for (int r = nvalid + (int)threadIdx.x; r < 2048; r += blockDim.x) ds[r] = 0;
}

}  // namespace mr

using namespace mr;

extern "C" int mr_ctu_search_noalloc(const mr_frame* cur, const mr_frame* ref,
                                     const mr_search_params* p, const uint8_t* bounds,
                                     const mr_mv_seed* seed, mr_search_out* out,
                                     void* hip_stream) {
  hipStream_t st = (hipStream_t)hip_stream;
  Plan P;
  P.defer_tables = true;
  const mr_search_out* o = out;
  int rc = make_plan(&cur, &ref, &p, &bounds, &o, &seed, 1, false, &P);
  if (rc != MR_OK) return rc;
  JobDesc& jb = P.jobs[0];
  const bool full = jb.seed_mv == nullptr;  // the full (or bounded) search needs key tables
  const int steps = full ? (jb.ntasks + kWaveSteps - 1) / kWaveSteps : 0;
  const size_t head = up256(sizeof(JobDesc)) + kCounterBytes;  // descriptor, queue counters
  const size_t qbytes = up256((size_t)steps * kWaveSteps * 4 * jb.D * 4);
  const size_t dbytes = up256((size_t)steps * 2048 * 8);
  if (head + qbytes + dbytes + P.scratch_bytes > kNoAllocBytes) return MR_ESCRATCH;
  uint8_t* base = nullptr;
  rc = noalloc_scratch(&base);
  if (rc != MR_OK) return rc;
  JobDesc* jobs_d = (JobDesc*)base;
  uint32_t* counter = (uint32_t*)(base + up256(sizeof(JobDesc)));
  hipError_t e = hipSuccess;
  if (full) {
    uint32_t* q = (uint32_t*)(base + head);
    uint64_t* d = (uint64_t*)(base + head + qbytes);
    jb.qtab = q;
    jb.dtab = d;
    hipLaunchKernelGGL(key_table_kernel, dim3(steps), dim3(256), 0, st, jb.R, jb.D, jb.Q,
                       jb.ntasks, jb.s, q, d);
    e = hipGetLastError();
  }
  bind_scratch(P, base + head + qbytes + dbytes);
  if (e == hipSuccess) e = launch_store_job(P.jobs[0], jobs_d, st);
  if (e == hipSuccess)
    e = launch_plan(P, jobs_d, nullptr, PlanLists{nullptr, nullptr, nullptr, nullptr}, counter, st,
                    nullptr);
  return e == hipSuccess ? MR_OK : MR_EHIP;
}
