// Device helpers shared by the compositing kernels.
#pragma once

#include "common.hpp"

namespace mgs {

constexpr int MAXB = 256;  // largest LDS batch of entries

struct TileGeom {
    int vi;
    int tx0, ty0;  // first pixel of the tile
};

__device__ __forceinline__ TileGeom tile_geom(const ViewSet& views, uint32_t tile, int TW, int TH) {
    TileGeom tg;
    int vi = 0;
    while (vi + 1 < views.n_views && tile >= views.v[vi + 1].tile_off) ++vi;
    tg.vi = vi;
    const DevView& cam = views.v[vi];
    const uint32_t lt = tile - cam.tile_off;
    tg.tx0 = (int)(lt % (uint32_t)cam.grid_w) * TW;
    tg.ty0 = (int)(lt / (uint32_t)cam.grid_w) * TH;
    return tg;
}

// Evaluation of one entry at one pixel, shared by forward and backward so
// both take the same FP32 decisions (3-sigma cut, alpha clamp and filter).
struct Eval {
    float dx, dy, t, G, oG, alpha;  // t = dx + beta dy
};

__device__ __forceinline__ bool eval_entry(const float4& A, const float4& B, float px, float py,
                                           const DevSettings& st, Eval& e) {
    e.dx = A.x - px;
    e.dy = A.y - py;
    e.t = fmaf(A.w, e.dy, e.dx);
    const float Q = A.z * e.t * e.t + B.x * e.dy * e.dy;
    if (!(Q <= st.q_max)) return false;
    e.G = __expf(-0.5f * Q);
    e.oG = B.y * e.G;
    e.alpha = fminf(st.alpha_max, e.oG);
    return e.alpha >= st.alpha_min;
}

// Persistent launches pop tile ids from a device counter; plain launches
// own tile blockIdx.x.
__device__ __forceinline__ uint32_t next_tile(uint32_t* queue, uint32_t* s_tile, uint32_t fixed) {
    if (!queue) return fixed;
    __syncthreads();
    if (threadIdx.x == 0) *s_tile = atomicAdd(queue, 1u);
    __syncthreads();
    return *s_tile;
}

// Workgroups a persistent launch needs to fill the device: resident blocks
// per CU at the kernel's register and LDS use, times the CU count.
template <typename Kernel>
inline int persistent_grid(Kernel k, int block, int num_cus, size_t dyn_lds = 0) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, block, dyn_lds) != hipSuccess || per_cu <= 0)
        per_cu = 4;
    return per_cu * num_cus;
}

}  // namespace mgs
