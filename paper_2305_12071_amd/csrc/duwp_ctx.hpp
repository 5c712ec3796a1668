// Host-side context of the DUWP library (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "duwp.h"
#include "duwp_device.hpp"

namespace duwp {

// One kernel of the step, for per-kernel timing.
struct KernelTimer {
    std::vector<std::string> names;
    std::vector<hipEvent_t> ev;     // ev[2*i], ev[2*i+1] bracket kernel i
    std::vector<double> ms;
    bool on = false;
    int idx = 0;
};

}  // namespace duwp

struct duwp_ctx {
    int ncases = 0, G = 0;
    int precision = DUWP_FP64;
    int use_graph = 0;
    int block_cells = 256;
    hipStream_t stream = nullptr;
    bool own_stream = false;  // created by the library when the caller passed none
    hipStream_t stream2 = nullptr;   // second stream for work independent of the collisions
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    uint64_t seed = 0;
    std::vector<duwp_case> cases;
    std::vector<duwp::DCase> hcases;
    int64_t cap = 0;          // particle capacity (canonical and staging arrays)
    int64_t inj_total = 0;    // injection buffer slots
    uint32_t step = 0;        // host copy of the step index
    int64_t avg_count = 0;

    duwp::DCase *d_cases = nullptr;
    void *A[2] = {nullptr};        // canonical particle records (x,u,v,w), by step parity
    void *S = nullptr;             // staging (intermediate) records
    void *J[4] = {nullptr};        // injected entrants
    int32_t *j_dest = nullptr, *j_rank = nullptr, *j_count = nullptr;
    void *K[4] = {nullptr};        // injection candidates
    int32_t *k_dest = nullptr;
    int64_t *k_n = nullptr;        // [ncases*2] candidates per side
    int64_t cand_total = 0;
    int32_t *k_chunk = nullptr;    // entrants per candidate chunk
    void *d_inj = nullptr;         // the entrant buffers' addresses (Inj<T>) for the scatter's entrant blocks
    int64_t chunk_total = 0;
    int32_t *hist_buf[2] = {nullptr, nullptr};   // destination histograms, by step parity
    int inj_blocks = 0;            // x-blocks of the candidate kernel
    int64_t *off[2] = {nullptr, nullptr};
    duwp::Cells cl{};
    int64_t *scan_part = nullptr;
    int ntiles = 0;
    uint32_t *d_step = nullptr;
    int32_t *d_err = nullptr;
    int64_t *d_nout = nullptr;     // [ncases]
    int64_t *d_ninj = nullptr;     // [ncases*2]
    int64_t *d_total = nullptr;    // [3] staged particles, next particle count, collision candidates
    int32_t *item_cell = nullptr;  // first cell of each collision work item
    int64_t *d_items = nullptr;    // [2] number of collision work items, candidates per item
    int64_t items_cap = 0;
    int coll_blocks = 0;
    int big_blocks = 0;            // grid of the block-per-cell collision kernel
    int rank_sep = 0;              // 1: the entrants are ranked by a kernel of their own (many candidates a side)
    int scat_by_order = 1;         // scatter blocks take cells largest first (few rounds of blocks)
    int abs_stream = 0;            // some case lets absorbed particles stream for their free time
    double *diag = nullptr;        // [G*5] on-demand cell diagnostics
    int64_t *d_psteps = nullptr;   // particle-steps since init or the last reset

    // tile shapes and thresholds (defaults filled in)
    int scat_items = 4;            // particles per thread and chunk, multi-wave scatter blocks
    int big_block = 512;           // threads of the block-per-cell collide
    int big_per_cu = 2;            // its resident blocks per compute unit
    int big_min_n = 4096, big_min_m = 4096;   // cells at least this large collide in it
    int coll_by_cell_max = 8192;   // up to this many cells: a wave per cell in k_collide
    int count_dests = 256;         // destinations per block of k_count_bases (large grids)

    hipGraphExec_t graph[2] = {nullptr, nullptr};
    bool graph_ready = false;
    duwp::KernelTimer timer;
    // device memory provider: the caller's, or hipMalloc/hipFree when alloc_fn is null
    void *(*alloc_fn)(size_t, void *) = nullptr;
    void (*free_fn)(void *, void *) = nullptr;
    void *alloc_ctx = nullptr;
    std::vector<void *> allocs;
    double *scratch = nullptr;     // this device's staging array of duwp_moments_noalloc
};

namespace duwp {
// Launch the kernels of one step on ctx->stream (defined with the kernels).
void enqueue_step(duwp_ctx *ctx);
// Scatter blocks that fit on one compute unit at once (for this precision, block size
// and items per thread of multi-wave blocks).
int scatter_blocks_per_cu(int precision, int bc, int items);
// Particle moments of cells [g0, g1) of the current canonical state: recomputed
// from the particles, or (recompute false) kept as loaded and checked for finite
// totals; then the destination histogram of the same cells (no averaging).
void enqueue_moments(duwp_ctx *ctx, int g0, int g1, bool recompute);
// Add delta to the canonical offsets off[g0..G].
void enqueue_shift_offsets(duwp_ctx *ctx, int64_t *off, int g0, int64_t delta);
// Normal stress and heat flux of cells [g0, g1) of the current state into out[G*5].
void enqueue_stress_heat(duwp_ctx *ctx, int g0, int g1, double *out);
// Device address of the staging array of duwp_moments_noalloc on device dev (taken
// once per device, with that device current).
hipError_t noalloc_setup(int dev, double **ptr);
}  // namespace duwp
