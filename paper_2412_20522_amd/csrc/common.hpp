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
    uint32_t wide_min;  // records covering more tiles than this are listed per region, not per tile
    int32_t reg_w, reg_h;  // region grid (REGION x REGION tiles per region)
    uint32_t reg_off;      // first region id of this view (region keys follow all tile keys)
};

// Passed by value as a kernel argument: no device copy, nothing to capture.
struct ViewSet {
    int32_t n_views;
    uint32_t total_tiles;
    uint32_t total_regions;
    DevView v[MGS_MAX_VIEWS];
};

// Effective constants (exact mode already folded in by the host).
struct DevSettings {
    int32_t tile_w, tile_h, batch, sh_degree;
    float alpha_min, alpha_max, t_min, q_max;
    float near_plane, dilation, lambda_floor;
    float bg[3];
    int32_t full_rect;  // every valid record covers every tile of its view
    int32_t tile_cull;  // narrow instances only for tiles a record can reach
    float qs_max;       // -log2(e) / 2 * q_max: the cut on the scaled form of the compositing kernels
    int32_t mask_opacity;  // 1: M multiplies the opacity in the projection (records carry mask 1)
};

// Side of a region in tiles.  Wide records are listed once per region they
// can reach instead of once per tile.
constexpr int REGION = 4;

// Device flag bits.
constexpr uint32_t FLAG_CAPACITY = 1u;
constexpr uint32_t FLAG_NONFINITE = 2u;

// Record layout: 3 float4 per (view, Gaussian) record.
//   A = (u, v, a, beta)
//   B = (gamma, opacity, mask, radius)
//   C = (r, g, b, number of tiles of the footprint as u32 bits)
// The conic (inverse 2D covariance, Q = a dx^2 + 2 b dx dy + c dy^2) is kept
// as a, beta = b / a and gamma = c - b^2 / a, so that
// Q = a (dx + beta dy)^2 + gamma dy^2 is a sum of two non-negative terms:
// FP32 evaluation of the expanded form loses every digit for needle-shaped
// splats (a c - b^2 tiny against a c), this one keeps full relative
// precision.  The per-record conic gradients refer to the stored
// (a, beta, gamma) as well.
constexpr int REC_F4 = 3;
// Per-record 2D gradient layout: du, dv, da, dbeta, dgamma, dopacity, dr, dg, db.
constexpr int DREC = 9;

// Tile rectangle (inclusive) of a record's square footprint; the same
// double-precision arithmetic as the tile count of the projection.
struct Rect {
    int x0, y0, x1, y1;
};

__device__ __forceinline__ Rect rect_of(float u, float v, float radius, const DevView& cam, const DevSettings& st) {
    Rect q;
    if (st.full_rect) {
        q.x0 = 0; q.y0 = 0; q.x1 = cam.grid_w - 1; q.y1 = cam.grid_h - 1;
        return q;
    }
    const double ud = u, vd = v, rd = radius;
    // tile sizes are powers of two: scaling by 2^-k is exact, so it equals
    // the FP64 division by the tile size
    const int kw = __builtin_ctz((unsigned)st.tile_w), kh = __builtin_ctz((unsigned)st.tile_h);
    const double fx0 = floor(ldexp(ud - rd, -kw)), fx1 = floor(ldexp(ud + rd, -kw));
    const double fy0 = floor(ldexp(vd - rd, -kh)), fy1 = floor(ldexp(vd + rd, -kh));
    // clamp into the grid before converting (values can be far outside it)
    q.x0 = (int)fmin(fmax(fx0, 0.0), (double)cam.grid_w);
    q.y0 = (int)fmin(fmax(fy0, 0.0), (double)cam.grid_h);
    q.x1 = (int)fmax(fmin(fx1, (double)(cam.grid_w - 1)), -1.0);
    q.y1 = (int)fmax(fmin(fy1, (double)(cam.grid_h - 1)), -1.0);
    return q;
}

__device__ __forceinline__ Rect record_rect(const float4* __restrict__ rec, const float* __restrict__ radius,
                                            int64_t r, const DevView& cam, const DevSettings& st) {
    const float4 A = rec[3 * r];
    return rect_of(A.x, A.y, radius[r], cam, st);
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    const int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Inclusive prefix sum over the 64 lanes of a wave with DPP row operations:
// shifts by 1, 2, 4 and 8 lanes within each 16-lane row (a lane with no
// source adds 0), then lane 15's sum into rows 1 and 3 and lane 31's into
// rows 2 and 3.  Lane 63 ends with the wave's total.
__device__ __forceinline__ uint32_t wave_add_scan(uint32_t v) {
    int x = (int)v;
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);  // row_shr 1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);  // row_shr 2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);  // row_shr 4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);  // row_shr 8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);  // row_bcast 15
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);  // row_bcast 31
    return (uint32_t)x;
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

// Maximum over the 64 lanes of a wave of non-negative values, with the
// pattern of wave_sum (lanes a DPP step leaves out contribute 0).
__device__ __forceinline__ float wave_max(float v) {
    int x = __float_as_int(v);
    v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0xb1, 0xf, 0xf, false)));
    x = __float_as_int(v);
    v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x4e, 0xf, 0xf, false)));
    x = __float_as_int(v);
    v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x124, 0xf, 0xf, false)));
    x = __float_as_int(v);
    v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x128, 0xf, 0xf, false)));
    x = __float_as_int(v);
    v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false)));
    x = __float_as_int(v);
    v = fmaxf(v, __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false)));
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
