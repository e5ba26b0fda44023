// Device-side types and wave64 primitives shared by the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "maskgs.h"

namespace mgs {

// One camera as the kernels see it (built on the host from mgs_camera).
struct DevView {
    float W[9];        // world -> camera rotation, row-major
    float t[3];        // world -> camera translation
    float fx, fy, cx, cy;
    float campos[3];   // camera centre in world space
    float limx, limy;  // lateral clamp of the EWA Jacobian
    int32_t width, height;
    int32_t grid_w, grid_h;
    uint32_t tile_off;  // first global tile id of this view
    uint32_t px_off;    // first pixel of this view in packed per-pixel arrays
};

// Passed by value as a kernel argument: no device copy, nothing to capture.
struct ViewSet {
    int32_t n_views;
    uint32_t total_tiles;
    DevView v[MGS_MAX_VIEWS];
};

// Effective constants (exact mode already folded in by the host).
struct DevSettings {
    int32_t tile_w, tile_h, batch, sh_degree;
    float alpha_min, alpha_max, t_min, q_max;
    float near_plane, dilation, lambda_floor;
    float bg[3];
    int32_t full_rect;  // every valid record covers every tile of its view
};

// Device flag bits.
constexpr uint32_t FLAG_CAPACITY = 1u;
constexpr uint32_t FLAG_NONFINITE = 2u;

// Record layout: 3 float4 per (view, Gaussian) record.
//   A = (u, v, conic a, conic b)
//   B = (conic c, opacity, mask, 0)
//   C = (r, g, b, 0)
constexpr int REC_F4 = 3;
// Per-record 2D gradient layout: du, dv, da, db, dc, dopacity, dr, dg, db.
constexpr int DREC = 9;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Sum over the 64 lanes of a wave with DPP row operations (GCN/CDNA row
// broadcast); the total lands in lane 63 and is returned to every lane.
__device__ __forceinline__ float wave_sum(float v) {
    int x = __float_as_int(v);
    // quad_perm [1,0,3,2] and [2,3,0,1]
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0xb1, 0xf, 0xf, false));
    x = __float_as_int(v);
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x4e, 0xf, 0xf, false));
    x = __float_as_int(v);
    // row_ror 4 and 8: every lane of a 16-lane row holds the row sum
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x124, 0xf, 0xf, false));
    x = __float_as_int(v);
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x128, 0xf, 0xf, false));
    x = __float_as_int(v);
    // row_bcast 15 into rows 1 and 3, then row_bcast 31 into rows 2 and 3
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false));
    x = __float_as_int(v);
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

__device__ __forceinline__ double block_sum_double(double v, double* sh) {
    // 256-thread block: wave partials through LDS, deterministic order.
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
    }
    return s;  // valid in thread 0
}

}  // namespace mgs
