// Host-side runtime of libmr: search layouts, key tables, job descriptors.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "mr.h"
#include "mr_internal.h"

namespace mr {

// sqrt(lambda) in Q16 with lambda = 0.57 * 2^((qp - 12) / 3).
int64_t sqrt_lambda_q16(int qp);
// Bits of the signed Exp-Golomb code of v.
int se_bits(int v);

// Tile choice of the search kernel for one job.
struct TileConfig {
  int D;        // vertical shifts per lane (2, 4 or 8)
  int nbands;   // dy bands the window is split into (1..kMaxBands)
};
TileConfig default_tiles(int R, int n_ctus);
SearchLayout make_layout(int R, const TileConfig& tc);

// Device tables of the rank-ordered arg-min keys for (qp, R, tiles); cached per device.
struct KeyTables {
  const uint32_t* qtab;
  const uint64_t* dtab;
};
int get_key_tables(int qp, const SearchLayout& L, KeyTables* out);

// Scratch bytes a job needs (curpack + keys + elig), 256-byte aligned pieces.
size_t job_scratch_bytes(int n_ctus);

// Fill a JobDesc from validated arguments and a scratch block.
void fill_job(JobDesc* jb, const mr_frame* cur, const mr_frame* ref, const mr_search_params* p,
              const uint8_t* bounds, const mr_search_out* out, const SearchLayout& L,
              const KeyTables& kt, void* scratch);

int validate_search(const mr_frame* cur, const mr_frame* ref, const mr_search_params* p,
                    const mr_search_out* out);

// Kernel launches (defined with the kernels).
hipError_t launch_prep1(const JobDesc& jb, hipStream_t st);
hipError_t launch_search1(const JobDesc& jb, size_t lds_bytes, hipStream_t st);
hipError_t launch_leaf1(const JobDesc& jb, hipStream_t st);
hipError_t launch_depth_bounds(const uint8_t* ref_depth, int ref_w, int ref_h, int dep_w,
                               int dep_h, int dlo, int dhi, uint8_t* out, hipStream_t st);

size_t search_lds_bytes(const SearchLayout& L);

}  // namespace mr
