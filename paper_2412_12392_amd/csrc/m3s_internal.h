// Host-side launchers of the gfx950 kernels (internal to libm3s).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "m3s_device.h"

namespace m3s {

// Tile configurations of the forward kernels (query tile TX x TY, one lane per query):
// 0: 32x8, 1: 16x16, 2: 64x4 with the refine reading global memory;
// 3: 16x16, 4: 32x8 with the refine region staged in LDS (D = 24 only);
// 5: 16x16 with an fp16 copy of the region and an exact fp32 rescoring of the
// candidates that can be the maximum (D = 24, r <= 5); 6: the same with 8x8
// one-wave tiles (64 lanes, no cross-wave barriers, 256-pixel regions).
constexpr int kNumTileConfigs = 7;
constexpr int kDefaultTileConfig = 5;
void tile_shape(int tile_config, int* tx, int* ty);
bool tile_uses_lds(int tile_config);

// Fallback-path counters kept on the device (indices match M3S_PATH_* of m3s.h).
enum { kPathLmGlobal = 0, kPathRefineGlobal = 1, kPathRefineQuery = 2, kPathBwdDirect = 3, kPathRefineBands = 4,
       kNumPathCounters = 8 };
// Synchronises the device, copies the counters to out[kNumPathCounters], optionally zeroes them.
hipError_t read_path_counters(int64_t* out, bool reset);

// Optional per-kernel event timing (implemented in m3s_capi.hip).  Both calls
// are no-ops unless timing is enabled and the stream is not being captured.
void timer_begin(const char* name, hipStream_t s);
void timer_end(hipStream_t s);

// Ray-record prep: one workgroup of 256 lanes per kPrepTX x kPrepTY pixels.
constexpr int kPrepTX = 32, kPrepTY = 8;
inline int64_t prep_tiles(int H, int W) {
    return (int64_t)((W + kPrepTX - 1) / kPrepTX) * (int64_t)((H + kPrepTY - 1) / kPrepTY);
}
hipError_t launch_prep(const float* Xii, float4* rays, int H, int W, hipStream_t s);
hipError_t launch_fwd(const EdgeArgs& A, int tile_config, bool desc_regs, bool xcd_remap, hipStream_t s);
// Ray-window margins and LM unroll factors of the persistent fp16 kernel
// (tile configuration 5); other configurations use the defaults.
constexpr int kMarginMin = 1, kMarginMax = 3, kDefaultMargin = 2, kUnrollMax = 2;
hipError_t launch_batched(const EdgeArgs* table, const int32_t* prep_begin, int n_edges, int total_prep_blocks,
                          int total_tiles, int32_t* counter, int tile_config, int grid, int margin, int unroll,
                          int levels, bool desc_regs, hipStream_t s);
// Device copy of `bytes` (a multiple of 4, both pointers 4-byte aligned)
// from pinned host memory, by a kernel on stream s.
hipError_t launch_host_copy(void* dst, const void* pinned_src, size_t bytes, hipStream_t s);
hipError_t launch_stats(const int32_t* idx, const uint8_t* valid, int H, int W, uint32_t* bitmap, int32_t* counts,
                        hipStream_t s);
// Backward of one edge: 16 x 16 query tiles (tiles_x x tiles_y), tile ids of
// the batched launch start at tile_begin.
struct BwdEdgeArgs {
    int32_t H, W, tiles_x, tiles_y, tile_begin;
    const float* Xii;
    const float* Xji;
    const float* p;
    const uint8_t* valid;
    const float* grad_p;
    const float* grad_xhat;        // may be nullptr
    float* dXii;
    float* dXji;
};
hipError_t launch_bwd(const BwdEdgeArgs& B, hipStream_t s);
// Zero every edge's dXii (one launch), then the backward over all edges'
// tiles with `grid` workgroups (one launch).  max_pixels: the largest H * W of
// the table.
hipError_t launch_bwd_batched(const BwdEdgeArgs* table, int n_edges, long max_pixels, int total_tiles, int grid,
                              bool zero, hipStream_t s);

// Tracking pose solve (m3s_track.hip): workgroups of one iteration launch,
// workspace bytes, and the launch sequence (init + iters + 1 launches).
int track_blocks(int N);
size_t track_workspace_bytes(int N);
hipError_t launch_track(int N, const float* Xk, const float* Xf, const int32_t* idx, const uint8_t* valid,
                        const float* Qf, const float* Qk, float q_min, float sigma_ray, float sigma_dist, float huber,
                        int iters, float* T, float* info, void* ws, hipStream_t s);
// Canonical pointmap fusion (Eq. 8) with the pose T read from device memory.
hipError_t launch_fuse(int N, const float* T, float* Xc, float* Cc, const float* X, const float* C, hipStream_t s);

// Backend Gauss-Newton (m3s_backend.hip).
int backend_blocks_per_edge(int HW);
size_t backend_workspace_bytes(int N, int HW, int E);
hipError_t launch_backend(int N, int HW, int E, const float* Xc, const float* Q, const int32_t* edges,
                          const int32_t* idx, const uint8_t* valid, float q_min, float sigma_ray, float sigma_dist,
                          float huber, int iters, double step_tol, float* T, float* info, void* ws, hipStream_t s);

}  // namespace m3s
