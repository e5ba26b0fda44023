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

// Entries staged in LDS hold a and gamma multiplied by QSCALE = -log2(e) / 2,
// so the Gaussian weight exp(-Q / 2) is exp2 of the staged quadratic form
// and the cut Q <= q_max reads qs >= QSCALE q_max (DevSettings::qs_max).
constexpr float QSCALE = -0.72134752044448170f;
// -1 / QSCALE = 2 ln 2
constexpr float QSCALE_NINV = 1.38629436111989061f;

__device__ __forceinline__ float4 stage_a(float4 A) {
    A.z *= QSCALE;
    return A;
}
__device__ __forceinline__ float4 stage_b(float4 B) {
    B.x *= QSCALE;
    return B;
}

// Per-kernel constants of the evaluation.
struct EvalConsts {
    float qs_max, amax, amin;
};
__device__ __forceinline__ EvalConsts eval_consts(const DevSettings& st) {
    return EvalConsts{st.qs_max, st.alpha_max, st.alpha_min};
}

// Evaluation of one staged entry at one pixel, shared by forward and
// backward so both take the same FP32 decisions (3-sigma cut, alpha clamp and
// filter).  A = (u, v, a', beta), B = (gamma', opacity, mask, .) with
// a' = QSCALE a and gamma' = QSCALE gamma.
struct Eval {
    float dy, t, apt, gdy, G, oG, alpha;  // t = dx + beta dy, apt = a' t, gdy = gamma' dy
};

__device__ __forceinline__ bool eval_entry(const float4& A, const float4& B, float px, float py,
                                           const EvalConsts& k, Eval& e) {
    const float dx = A.x - px;
    e.dy = A.y - py;
    e.t = fmaf(A.w, e.dy, dx);
    e.apt = A.z * e.t;
    e.gdy = B.x * e.dy;
    const float qs = fmaf(e.apt, e.t, e.gdy * e.dy);  // QSCALE Q <= 0
    // computed for every pair, so that alpha needs no select on the cut
    e.G = __builtin_amdgcn_exp2f(qs);
    e.oG = B.y * e.G;
    // min(alpha_max, oG) for oG >= 0 in one instruction (a min would first
    // canonicalise its operands)
    e.alpha = __builtin_amdgcn_fmed3f(e.oG, 0.f, k.amax);
    return (qs >= k.qs_max) & (e.alpha >= k.amin);
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
