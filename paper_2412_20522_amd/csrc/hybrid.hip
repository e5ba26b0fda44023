// Hybrid binning and compositing for scenes with screen-covering splats.
//
// A record whose tile footprint exceeds a per-view threshold ("wide") is not
// duplicated into every tile it covers but into every region (REGION x
// REGION tiles) its footprint overlaps; the remaining ("narrow") records are
// duplicated per tile.  Both kinds of entry share one key space (tile ids,
// then region ids) and one stable sort, so each tile and each region holds
// its entries in (depth, record) order.  A tile's list in the sense of
// Sec. 3.1 -- every record whose footprint covers the tile, in depth order --
// is then the merge of the tile's narrow entries with the entries of its
// region whose rectangle contains the tile.  The compositing kernels form
// that merged list batch by batch in LDS (merge path over two ordered
// windows), so the entries, their order and the per-pixel results are
// exactly those of fully duplicated lists, while the instance sort shrinks
// from every (tile, wide splat) pair to one entry per region.
//
// With culling, an entry is kept only where the splat can pass the per-pixel
// filters at some pixel centre of the cell (exact test, conservative
// margin): narrow entries per tile at duplication, wide entries per region
// at duplication and per tile before the merge.  Dropped entries contribute
// nothing to any pixel; the merged lists are shorter, the results the same.
//
// Records are copied once into (view, depth, record) order ("sorted
// records"); list entries hold positions in that order, which are unique and
// order exactly as (depth, record) within a view, so the merge compares plain
// 32-bit positions and the record gathers of a tile walk memory upwards.
//
// The forward records, per tile and batch, the stream cursors where the batch
// began; the backward replays the same batches in reverse from those
// checkpoints, so the merge is deterministic and nothing per pixel beyond the
// final transmittance and the last blended entry is stored.
#include "common.hpp"
#include "composite_common.hpp"
#include "kernels.hpp"

namespace mgs {
namespace {

// The tile's pixel centres span [X0, X1] x [Y0, Y1].
struct TileBox {
    float X0, X1, Y0, Y1;
};

// Whether an entry can pass the per-pixel filters (Q <= q_max and
// alpha >= alpha_min) at any pixel centre of the tile: the minimum of its
// quadratic form over the box (zero if the centre is inside, else the
// smallest of the clamped minima along the four edges) against the cut
// min(q_max, 2 ln(opacity / alpha_min)).  The test is conservative (a small
// margin over the cut), so an entry it drops contributes nothing to any
// pixel of the tile in the forward or the backward pass; dropping it leaves
// every result unchanged.
struct TouchPrep {
    float u, v, a, beta, gamma;
    float nbc;       // -b / c: minimiser along a vertical edge (-beta along a horizontal one)
    float cut;       // +huge: no cut (always touches); < 0: reaches no pixel
};

// Every operation below is written out (fmaf where a fused product is meant)
// and contraction is off, so the rounding of each step is fixed by the
// source: the binning kernels inline the test and still take identical
// decisions for the same record and cell.
__device__ __forceinline__ TouchPrep touch_prep(const float4& A, const float4& B, float q_max, float alpha_min) {
#pragma clang fp contract(off)
    TouchPrep p;
    p.u = A.x;
    p.v = A.y;
    p.a = A.z;
    p.beta = A.w;
    p.gamma = B.x;
    // -b / c = -a beta / (a beta^2 + gamma); a reciprocal approximation only
    // moves the edge minimiser slightly, which raises the computed minimum by
    // a second-order amount far inside the margin below
    const float ab = p.a * p.beta;
    p.nbc = -ab * __builtin_amdgcn_rcpf(fmaf(ab, p.beta, p.gamma));
    float cut = q_max;
    if (alpha_min > 0.f) cut = fminf(cut, 2.f * __logf(B.y / alpha_min));
    if (cut >= 3.0e38f) p.cut = 3.4e38f;          // no finite cut
    else if (!(cut > -3.0e38f)) p.cut = -1.f;     // zero opacity
    else p.cut = fmaf(1e-3f, 1.f + fabsf(cut), cut);
    return p;
}

__device__ __forceinline__ TouchPrep touch_prep(const float4& A, const float4& B, const DevSettings& st) {
    return touch_prep(A, B, st.q_max, st.alpha_min);
}

// a (dx + beta dy)^2 + gamma dy^2
__device__ __forceinline__ float touch_q(const TouchPrep& p, float dx, float dy) {
#pragma clang fp contract(off)
    const float t = fmaf(p.beta, dy, dx);
    const float at = p.a * t;
    const float gdy = p.gamma * dy;
    return fmaf(at, t, gdy * dy);
}

__device__ __forceinline__ bool touch_test(const TouchPrep& p, const TileBox& tb) {
#pragma clang fp contract(off)
    if (p.cut >= 3.0e38f) return true;  // no cut (exact mode)
    if (p.cut < 0.f) return false;
    if (p.u >= tb.X0 && p.u <= tb.X1 && p.v >= tb.Y0 && p.v <= tb.Y1) return true;
    const float dyl = p.v - tb.Y1, dyh = p.v - tb.Y0, dxl = p.u - tb.X1, dxh = p.u - tb.X0;
    // along the vertical edges dy minimises at -b/c dx, along the horizontal
    // ones dx at -beta dy, each clamped to the edge
    float q = touch_q(p, dxh, fminf(fmaxf(p.nbc * dxh, dyl), dyh));
    q = fminf(q, touch_q(p, dxl, fminf(fmaxf(p.nbc * dxl, dyl), dyh)));
    q = fminf(q, touch_q(p, fminf(fmaxf(-p.beta * dyh, dxl), dxh), dyh));
    q = fminf(q, touch_q(p, fminf(fmaxf(-p.beta * dyl, dxl), dxh), dyl));
    return q <= p.cut;
}

__device__ __forceinline__ bool may_touch(const float4& A, const float4& B, const TileBox& tb,
                                          const DevSettings& st) {
    return touch_test(touch_prep(A, B, st), tb);
}

// Pixel-centre box of cell (cx, cy) of a grid of cw x ch pixel cells.
__device__ __forceinline__ TileBox cell_box(int cx, int cy, int cw, int ch, const DevView& cam) {
    const int x0 = cx * cw, y0 = cy * ch;
    return TileBox{(float)x0 + 0.5f, (float)min(x0 + cw, cam.width) - 0.5f, (float)y0 + 0.5f,
                   (float)min(y0 + ch, cam.height) - 0.5f};
}

// ---------------------------------------------------------------------------
// binning: (view, depth) order of records, sorted records, per-tile and
// per-region lists, batch checkpoints
// ---------------------------------------------------------------------------

// Depth keys of the records, sorted per view (the records of view v are the
// segment [v n, (v + 1) n)): the float bits of the view-space depth (positive,
// so the bits order like the values), all ones for a record without tiles,
// which sorts it after every listed record of its view.
// The cells a record is listed in: the tiles of its rectangle for a narrow
// record, the regions (REGION x REGION tiles) its rectangle overlaps for a
// wide one.  Cell j of the rectangle is (x0 + j % w, y0 + j / w).
struct Cells {
    int x0, y0, w;
    uint32_t area;   // 0: the record is listed nowhere
    int cw, ch;      // cell size in pixels
};

__device__ __forceinline__ Cells cells_of(const float4& A, const float4& B, bool wide, const DevView& cam,
                                          const DevSettings& st) {
    Cells c{0, 0, 1, 0u, st.tile_w, st.tile_h};
    const Rect q = rect_of(A.x, A.y, B.w, cam, st);
    if (q.x1 < q.x0 || q.y1 < q.y0) return c;
    if (wide) {
        c.x0 = q.x0 / REGION;
        c.y0 = q.y0 / REGION;
        c.w = q.x1 / REGION - c.x0 + 1;
        c.area = (uint32_t)c.w * (uint32_t)(q.y1 / REGION - c.y0 + 1);
        c.cw = REGION * st.tile_w;
        c.ch = REGION * st.tile_h;
    } else {
        c.x0 = q.x0;
        c.y0 = q.y0;
        c.w = q.x1 - q.x0 + 1;
        c.area = (uint32_t)c.w * (uint32_t)(q.y1 - q.y0 + 1);
    }
    return c;
}

// Sort key of cell (cx, cy): tile ids first, then region ids.
__device__ __forceinline__ uint32_t cell_key(bool wide, int cx, int cy, const DevView& cam, const ViewSet& views) {
    return wide ? views.total_tiles + cam.reg_off + (uint32_t)cy * (uint32_t)cam.reg_w + (uint32_t)cx
                : cam.tile_off + (uint32_t)cy * (uint32_t)cam.grid_w + (uint32_t)cx;
}

// Row-wise culling of the binning.  Within a band of pixel-centre rows
// [Y0, Y1] the points where an entry can pass the per-pixel filters form the
// band's slice of the ellipse a (ex + beta ey)^2 + gamma ey^2 <= cut (ex, ey
// offsets from the centre; cut = min(q_max, 2 ln(opacity / alpha_min)) plus a
// margin), and the slice's x-extent is an interval: the chord's right end
// -beta ey + sqrt((cut - gamma ey^2) / a) is concave in ey, so its maximum
// over the band is at the ellipse's rightmost point (ey = eyR) clamped to the
// band, and the left end's minimum at -eyR.  A cell of the row is kept iff
// the interval meets the cell's pixel-centre columns -- the decision of a
// test of the quadratic form's minimum over each cell's box, taken once per
// row.  Every operation is written out and contraction is off, so the
// classification (which counts) and the duplication (which emits) take
// identical decisions; culled cells contribute nothing to any pixel.
// Reciprocals and square roots are the hardware's single instructions (about
// one ulp): their error is orders of magnitude inside the margins (1e-3 of
// the cut, 1e-3 pixel), so the test stays conservative.
struct RowCull {
    float u, v, beta, gamma, inva, cut, H, eyR;
    int mode;  // 0: cull, 1: every cell (no finite cut), 2: no cell
};

__device__ __forceinline__ RowCull row_prep(const float4& A, const float4& B, const DevSettings& st) {
#pragma clang fp contract(off)
    RowCull p;
    p.u = A.x;
    p.v = A.y;
    p.beta = A.w;
    p.gamma = B.x;
    const float a = A.z;
    float cut = st.q_max;
    if (st.alpha_min > 0.f) cut = fminf(cut, 2.f * __logf(B.y / st.alpha_min));
    p.mode = 0;
    p.cut = 0.f;
    if (cut >= 3.0e38f) {
        p.mode = 1;
    } else if (!(cut > -3.0e38f)) {
        p.mode = 2;
    } else {
        p.cut = fmaf(1e-3f, 1.f + fabsf(cut), cut);
        if (!(p.cut >= 0.f)) p.mode = 2;
    }
    p.inva = __builtin_amdgcn_rcpf(a);
    p.H = __builtin_amdgcn_sqrtf(p.cut * __builtin_amdgcn_rcpf(p.gamma));
    const float D = fmaf(a * p.beta, p.beta, p.gamma);  // c = gamma + a beta^2
    p.eyR = -p.beta * __builtin_amdgcn_sqrtf(p.cut * a * __builtin_amdgcn_rcpf(p.gamma * D));
    return p;
}

// Columns [lo, hi] (within [x0, x1]) of cell row cy, cells of cw x ch pixels
// (powers of two), that the entry can reach; false if none.
__device__ __forceinline__ bool row_cells(const RowCull& p, int cy, int cw, int ch, int x0, int x1, int width,
                                          int height, int& lo, int& hi) {
#pragma clang fp contract(off)
    lo = x0;
    hi = x1;
    if (p.mode == 1) return true;
    if (p.mode == 2) return false;
    const float Y0 = (float)(cy * ch) + 0.5f, Y1 = (float)min((cy + 1) * ch, height) - 0.5f;
    const float e0 = fmaxf(Y0 - p.v, -p.H), e1 = fminf(Y1 - p.v, p.H);
    if (!(e0 <= e1)) return false;
    const float eR = fminf(fmaxf(p.eyR, e0), e1), eL = fminf(fmaxf(-p.eyR, e0), e1);
    const float gR = p.gamma * eR, gL = p.gamma * eL;
    const float sR = __builtin_amdgcn_sqrtf(fmaxf(0.f, (p.cut - gR * eR) * p.inva));
    const float sL = __builtin_amdgcn_sqrtf(fmaxf(0.f, (p.cut - gL * eL) * p.inva));
    const float xhi = p.u + (sR - p.beta * eR) + 1e-3f;
    const float xlo = p.u - (sL + p.beta * eL) - 1e-3f;
    if (!(xlo <= (float)width - 0.5f && xhi >= 0.5f)) return false;
    // cell cx spans pixel centres [cx cw + 0.5, (cx + 1) cw - 0.5]
    const float icw = ldexpf(1.f, -__builtin_ctz((unsigned)cw));  // exact: cw is a power of two
    const float flo = fmaxf(ceilf((xlo + 0.5f) * icw - 1.f), (float)x0);
    const float fhi = fminf(floorf((xhi - 0.5f) * icw), (float)x1);
    if (!(flo <= fhi)) return false;
    lo = (int)flo;
    hi = (int)fhi;
    return true;
}

// With culling, the kept cells of a rectangle of at most CULL_MAX cells
// travel from the classification to the duplication as a bit mask (bit j:
// cell j, row-major); larger rectangles have their rows recomputed.
constexpr uint32_t CULL_MAX = 64;
// Key of an emitted slot the duplication could not fill: past every cell,
// so it sorts last and no range includes it.
constexpr uint32_t KEY_NONE = 0xffffffffu;
// Bit of a position's entry count that marks a wide record (listed per
// region); the count itself is below 2^24.
constexpr uint32_t CNT_WIDE = 0x80000000u;

__device__ __forceinline__ float4 shfl4(const float4& v, int src) {
    return make_float4(__shfl(v.x, src), __shfl(v.y, src), __shfl(v.z, src), __shfl(v.w, src));
}

// Sorted position i holds record order[i] with depth key skeys[i]; positions
// [v n, (v + 1) n) belong to view v.  Writes the sorted record copy (radius in
// B.w, record id bits in C.w), the wide flag and the number of list entries
// (tiles or regions, after culling) of every position, and per workgroup the
// number of wide records and of their region entries (part[b], part[nb +
// b]), and per wave the number of all list entries (part[2 nb + wave]; a
// position has fewer than 2^24 entries, so a wave's 64 stay below 2^32).
// A record without tiles (key all ones, sorted last in its view) is listed
// nowhere: it gets no copy, which nothing uses.
__global__ void __launch_bounds__(256) permute_classify_kernel(
    const uint32_t* __restrict__ order, const uint32_t* __restrict__ skeys, const float4* __restrict__ rec,
    int64_t R, int64_t n, ViewSet views, DevSettings st, uint32_t* __restrict__ cnt_out,
    uint64_t* __restrict__ tmask, float4* __restrict__ srec,
    uint32_t* __restrict__ part) {
    __shared__ uint32_t s_part[2][4];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = lane_id();
    const bool live = i < R;
    float4 A = make_float4(0.f, 0.f, 0.f, 0.f), B = A;
    uint32_t c = 0;
    bool wide = false;
    int vi = 0;
    // both loads of the position in one round trip, then the record
    const uint32_t key = live ? skeys[i] : 0xffffffffu;
    const uint32_t r = live ? order[i] : 0u;
    if (live && key != 0xffffffffu) {
        // one gather of the record (radius in B.w, tile count in C.w)
        A = rec[3 * (size_t)r];
        B = rec[3 * (size_t)r + 1];
        uint4 C = reinterpret_cast<const uint4*>(rec)[3 * (size_t)r + 2];
        c = C.w;
        vi = (int)((uint32_t)i / (uint32_t)n);  // positions are below 2^32
        wide = c > views.v[vi].wide_min;
        C.w = r;
        srec[3 * i] = A;
        srec[3 * i + 1] = B;
        reinterpret_cast<uint4*>(srec)[3 * i + 2] = C;
    }
    Cells cl{0, 0, 1, 0u, st.tile_w, st.tile_h};
    if (live && c > 0) cl = cells_of(A, B, wide, views.v[vi], st);
    uint32_t cnt = cl.area;
    uint64_t mask = 0;
    if (st.tile_cull && cl.area > 0) {
        const RowCull rc = row_prep(A, B, st);
        const int width = views.v[vi].width, height = views.v[vi].height;  // loaded once, not per row
        const int rows = (int)(cl.area / (uint32_t)cl.w);
        cnt = 0;
        for (int ry = 0; ry < rows; ++ry) {
            int lo, hi;
            if (!row_cells(rc, cl.y0 + ry, cl.cw, cl.ch, cl.x0, cl.x0 + cl.w - 1, width, height, lo, hi)) continue;
            cnt += (uint32_t)(hi - lo + 1);
            if (cl.area <= CULL_MAX) {
                // bits ry w + (lo - x0) .. ry w + (hi - x0)
                const uint32_t b0 = (uint32_t)(ry * cl.w + (lo - cl.x0)), nb = (uint32_t)(hi - lo + 1);
                mask |= (nb >= 64 ? ~0ull : ((1ull << nb) - 1ull)) << b0;
            }
        }
    }
    if (live) {
        // the wide flag rides in bit 31 (counts stay below 2^24); the cull
        // mask is kept only for positions with entries
        cnt_out[i] = cnt | (wide ? CNT_WIDE : 0u);
        if (cnt != 0) tmask[i] = mask;
    }
    // wide records and their list entries of the workgroup (no atomics: one
    // address updated by every wave serialises)
    const uint64_t wb = __ballot(live && wide);
    // the wave's totals land in lane 63
    const uint32_t e = wave_add_scan(live && wide ? cnt : 0u);
    const uint32_t ea = wave_add_scan(live ? cnt : 0u);
    const int wid = threadIdx.x >> 6;
    if (lane == 63) {
        s_part[0][wid] = (uint32_t)__popcll(wb);
        s_part[1][wid] = e;
        part[2 * gridDim.x + (blockIdx.x * blockDim.x + threadIdx.x) / 64] = ea;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t a = 0, b = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            a += s_part[0][w];
            b += s_part[1][w];
        }
        part[blockIdx.x] = a;
        part[gridDim.x + blockIdx.x] = b;
    }
}

// List offsets from the classification's counts, in two steps.  A group is
// LO_GROUP waves (LO_GROUP / 4 classification workgroups).  Step 1, one
// workgroup per group: each wave's first entry relative to its group (an
// exclusive scan of the per-wave entry counts), the group's entry total and
// its totals of wide records and their region entries.  Step 2, one
// workgroup: the groups' first entries, the entry total (*total) and the
// wide totals (wide[0], wide[2]).  A wave's first entry is then
// wave_rel[wave] + group_off[wave / LO_GROUP].  Integer sums: no result
// depends on an order.
constexpr int LO_GROUP = 1024;
struct ListOffsets {
    uint64_t* wave_rel;   // [waves]
    uint64_t* group_tot;  // [groups, 3]: entries, wide records, region entries
    uint64_t* group_off;  // [groups]
};

__global__ void __launch_bounds__(LO_GROUP) list_offsets_group_kernel(const uint32_t* __restrict__ part, int64_t nb,
                                                                     int64_t nw, ListOffsets lo) {
    __shared__ uint64_t s_w[LO_GROUP / 64][3];
    const int t = threadIdx.x, lane = lane_id(), wid = t >> 6;
    const int64_t w = (int64_t)blockIdx.x * LO_GROUP + t;  // this thread's wave
    const uint64_t c = w < nw ? part[2 * nb + w] : 0u;
    // the group's classification workgroups: LO_GROUP / 4 of them
    const int64_t b = (int64_t)blockIdx.x * (LO_GROUP / 4) + t;
    uint64_t a = 0, r = 0;
    if (t < LO_GROUP / 4 && b < nb) {
        a = part[b];
        r = part[nb + b];
    }
    uint64_t x = c;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint64_t y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off);
        r += __shfl_xor(r, off);
    }
    if (lane == 63) s_w[wid][0] = x;
    if (lane == 0) {
        s_w[wid][1] = a;
        s_w[wid][2] = r;
    }
    __syncthreads();
    uint64_t wo = 0;
    for (int v = 0; v < wid; ++v) wo += s_w[v][0];
    if (w < nw) lo.wave_rel[w] = wo + x - c;
    if (t < 3) {
        uint64_t tot = 0;
        for (int v = 0; v < LO_GROUP / 64; ++v) tot += s_w[v][t];
        lo.group_tot[3 * blockIdx.x + t] = tot;
    }
}

__global__ void __launch_bounds__(LO_GROUP) list_offsets_total_kernel(int64_t ng, ListOffsets lo,
                                                                     uint64_t* __restrict__ total,
                                                                     uint64_t* __restrict__ wide) {
    __shared__ uint64_t s_w[LO_GROUP / 64][3];
    const int t = threadIdx.x, lane = lane_id(), wid = t >> 6;
    uint64_t carry = 0, a = 0, r = 0;
    for (int64_t base = 0; base < ng; base += LO_GROUP) {
        const int64_t g = base + t;
        const uint64_t c = g < ng ? lo.group_tot[3 * g] : 0u;
        if (g < ng) {
            a += lo.group_tot[3 * g + 1];
            r += lo.group_tot[3 * g + 2];
        }
        uint64_t x = c;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint64_t y = __shfl_up(x, d);
            if (lane >= d) x += y;
        }
        if (lane == 63) s_w[wid][0] = x;
        __syncthreads();
        uint64_t wo = 0, tot = 0;
        for (int v = 0; v < LO_GROUP / 64; ++v) {
            if (v < wid) wo += s_w[v][0];
            tot += s_w[v][0];
        }
        if (g < ng) lo.group_off[g] = carry + wo + x - c;
        carry += tot;
        __syncthreads();  // s_w is written again by the next round
    }
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off);
        r += __shfl_xor(r, off);
    }
    if (lane == 0) {
        s_w[wid][1] = a;
        s_w[wid][2] = r;
    }
    __syncthreads();
    if (t == 0) {
        uint64_t ta = 0, tr = 0;
        for (int v = 0; v < LO_GROUP / 64; ++v) {
            ta += s_w[v][1];
            tr += s_w[v][2];
        }
        *total = carry;
        wide[0] = ta;
        wide[2] = tr;
    }
}

// Position of the r-th (0-based) set bit of m; r < popcount(m).
__device__ __forceinline__ uint32_t select_bit(uint64_t m, uint32_t r) {
    uint32_t pos = 0;
    uint32_t x = (uint32_t)m;
    uint32_t c = (uint32_t)__popc(x);
    if (r >= c) {
        r -= c;
        x = (uint32_t)(m >> 32);
        pos = 32;
    }
#pragma unroll
    for (int sh = 16; sh >= 1; sh >>= 1) {
        c = (uint32_t)__popc(x & ((1u << sh) - 1u));
        if (r >= c) {
            r -= c;
            x >>= sh;
            pos += (uint32_t)sh;
        }
    }
    return pos;
}

// Inclusive maximum scan over the 64 lanes of a wave, for values >= -1:
// shifts within each 16-lane row, then the broadcasts of lane 15 into rows
// 1 and 3 and of lane 31 into rows 2 and 3 (a lane with no source keeps -1).
__device__ __forceinline__ int wave_max_scan(int x) {
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x111, 0xf, 0xf, false));  // row_shr 1
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x112, 0xf, 0xf, false));  // row_shr 2
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x114, 0xf, 0xf, false));  // row_shr 4
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x118, 0xf, 0xf, false));  // row_shr 8
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x142, 0xa, 0xf, false));  // row_bcast 15
    x = max(x, __builtin_amdgcn_update_dpp(-1, x, 0x143, 0xc, 0xf, false));  // row_bcast 31
    return x;
}

// List entries in sorted-position order: cell keys (tile or region ids) as
// keys, positions as values, for the cells the classification counted.  The
// outputs of a wave's records are contiguous, so each wave walks them 64
// slots at a time with every lane busy and consecutive lanes writing
// consecutive entries.  The owner of a slot is the last record whose first
// slot is at or before it: every record marks its first slot (records with
// entries start at distinct slots), and a running maximum over the slots
// fills the rest.  Record-local rank -> cell by selecting the rank-th bit of
// the cull mask (the rank itself without culling).  Culled rectangles of
// more than CULL_MAX cells re-derive their rows, one row per lane.  Writes
// never leave a record's counted slots; a slot the emission does not fill
// gets KEY_NONE.  No step waits on another wave.
__global__ void __launch_bounds__(256) duplicate_kernel(
    const float4* __restrict__ srec, const uint32_t* __restrict__ cnt_sorted,
    const uint64_t* __restrict__ tmask, ListOffsets lo, int64_t R, int64_t n, ViewSet views, DevSettings st,
    uint32_t* __restrict__ keys, uint32_t* __restrict__ vals, int64_t capacity, uint32_t* __restrict__ flags) {
    __shared__ uint32_t s_first[256];
    __shared__ uint32_t s_rel[256];
    __shared__ unsigned long long s_mask[256];
    __shared__ uint2 s_geo[256];
    __shared__ int s_own[256];
    const int t = threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x;
    const int64_t i = i0 + t;
    const int lane = lane_id();
    const int wb = t & ~63;  // the wave's first thread
    Cells cl{0, 0, 1, 0u, st.tile_w, st.tile_h};
    uint32_t cnt = 0;
    int vi = 0;
    bool wide = false;
    uint64_t mask = 0;
    float4 A = make_float4(0.f, 0.f, 0.f, 0.f), B = A;
    const bool cull = st.tile_cull != 0;
    if (i < R) {
        const uint32_t cw = cnt_sorted[i];
        cnt = cw & ~CNT_WIDE;
        wide = (cw & CNT_WIDE) != 0;
    }
    // the copy and the mask of a position without entries (never written)
    // are not used: positions listed nowhere sort last in their view, so
    // whole waves of them load nothing more
    if (__any(cnt != 0) && i < R) {
        A = srec[3 * i];
        B = srec[3 * i + 1];
        if (cull) mask = tmask[i];
    }
    // the record's view, loaded once: cell (x0 + rx, y0 + ry) has key
    // key0 + ry stride + rx
    uint32_t key0 = 0, stride = 0;
    int width = 0, height = 0;
    if (cnt != 0) {
        vi = (int)((uint32_t)i / (uint32_t)n);  // positions are below 2^32
        const DevView& cam = views.v[vi];
        cl = cells_of(A, B, wide, cam, st);
        key0 = cell_key(wide, cl.x0, cl.y0, cam, views);
        stride = (uint32_t)(wide ? cam.reg_w : cam.grid_w);
        width = cam.width;
        height = cam.height;
    }
    if (cnt == 0 || cl.area > CULL_MAX) mask = 0;
    const bool flat = cnt > 0 && (!cull || cl.area <= CULL_MAX);
    // start of the wave's output: its offset within its group of waves plus
    // the group's
    const int64_t wave = i0 / 64 + (t >> 6);
    const int64_t base = (int64_t)(lo.wave_rel[wave] + lo.group_off[wave / LO_GROUP]);
    bool overflow = false;
    // the record's first entry: the wave's start plus the entries of the
    // wave's earlier positions (below 2^32, see the classification)
    uint32_t rel;
    {
        // inclusive scans over the wave: all entries (ax), flat slots (x)
        const uint32_t x = wave_add_scan(flat ? cnt : 0u), ax = wave_add_scan(cnt);
        rel = ax - cnt;
        // first slot of each record among the wave's flat slots
        const uint32_t first = x - (flat ? cnt : 0u);
        const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
        s_first[t] = first;
        s_rel[t] = rel;
        s_mask[t] = mask;
        s_geo[t] = make_uint2(key0, (uint32_t)cl.w | (stride << 16));
        int carry = -1;
        for (uint32_t w0 = 0; w0 < total; w0 += 64) {
            // LDS operations of one wave complete in program order
            s_own[t] = -1;
            __builtin_amdgcn_wave_barrier();
            if (flat && first >= w0 && first < w0 + 64u) s_own[wb + (int)(first - w0)] = lane;
            __builtin_amdgcn_wave_barrier();
            const int own = max(wave_max_scan(s_own[t]), carry);
            carry = __builtin_amdgcn_readlane(own, 63);
            __builtin_amdgcn_wave_barrier();
            const uint32_t e = w0 + (uint32_t)lane;
            if (e >= total) continue;
            const int k = wb + own;
            const uint32_t r = e - s_first[k];
            const uint2 g = s_geo[k];
            const uint32_t w = g.y & 0xffffu, kstride = g.y >> 16;
            const uint64_t km = s_mask[k];
            const int64_t o = base + (int64_t)s_rel[k] + (int64_t)r;
            uint32_t key = KEY_NONE;
            if (!cull || r < (uint32_t)__popcll(km)) {
                const uint32_t j = cull ? select_bit(km, r) : r;
                // with culling j < 64 and w <= 64: (j + 1/2) / w is at least
                // 1/128 from an integer, far beyond the product's rounding
                const uint32_t ry = cull ? (uint32_t)(((float)j + 0.5f) * __builtin_amdgcn_rcpf((float)w)) : j / w;
                const uint32_t rx = j - ry * w;
                key = g.x + ry * kstride + rx;
            }
            if (o < capacity) {
                keys[o] = key;
                vals[o] = key == KEY_NONE ? 0u : (uint32_t)(i0 + k);
            } else {
                overflow = true;
            }
        }
    }
    // culled rectangles of more than CULL_MAX cells: the rows again, one row
    // per lane; each row is a contiguous run of cells placed by a prefix sum
    uint64_t pending = __ballot(cnt > 0 && !flat);
    while (pending) {
        const int src = __ffsll((long long)pending) - 1;
        pending &= pending - 1;
        const uint32_t barea = __shfl(cl.area, src), bcnt = __shfl(cnt, src);
        const uint32_t bi = (uint32_t)__shfl((int)(uint32_t)i, src);
        const int bx0 = __shfl(cl.x0, src), by0 = __shfl(cl.y0, src), bw = __shfl(cl.w, src);
        const int bcw = __shfl(cl.cw, src), bch = __shfl(cl.ch, src);
        const int bwidth = __shfl(width, src), bheight = __shfl(height, src);
        const uint32_t bkey0 = (uint32_t)__shfl((int)key0, src), bstride = (uint32_t)__shfl((int)stride, src);
        const int64_t bo = base + (int64_t)(uint32_t)__shfl((int)rel, src);
        const int64_t end = bo + bcnt;
        const RowCull rc = row_prep(shfl4(A, src), shfl4(B, src), st);
        const int rows = (int)(barea / (uint32_t)bw);
        int64_t rbase = bo;
        for (int r0 = 0; r0 < rows && rbase < end; r0 += 64) {
            const int ry = r0 + lane;
            int lo = 0, hi = -1;
            if (ry < rows && !row_cells(rc, by0 + ry, bcw, bch, bx0, bx0 + bw - 1, bwidth, bheight, lo, hi))
                hi = lo - 1;
            if (ry >= rows) hi = lo - 1;
            const int nrow = hi - lo + 1;
            int incl = nrow;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const int y = __shfl_up(incl, d);
                if (lane >= d) incl += y;
            }
            int64_t o = rbase + (incl - nrow);
            for (int cx = lo; cx <= hi && o < end; ++cx, ++o) {
                if (o < capacity) {
                    keys[o] = bkey0 + (uint32_t)ry * bstride + (uint32_t)(cx - bx0);
                    vals[o] = bi;
                } else {
                    overflow = true;
                }
            }
            rbase += __shfl(incl, 63);
        }
        for (int64_t o = rbase + lane; o < end; o += 64) {
            if (o < capacity) {
                keys[o] = KEY_NONE;
                vals[o] = 0u;
            } else {
                overflow = true;
            }
        }
    }
    if (overflow) atomicOr(flags, FLAG_CAPACITY);
}

// Upper bound on the batches a tile can take: a batch either emits `batch`
// merged entries or exhausts a whole window of one of the two streams.
__device__ __forceinline__ uint32_t region_of_tile(int tx, int ty, const DevView& cam, const ViewSet& views) {
    return views.total_tiles + cam.reg_off + (uint32_t)(ty / REGION) * (uint32_t)cam.reg_w + (uint32_t)(tx / REGION);
}

// Per tile: the batch checkpoints it may take (a batch either emits `batch`
// merged entries or exhausts a whole window of one of the two streams), as
// an exclusive prefix within the workgroup (cur_off) and the workgroup's
// total (blk); the forward's cost key (cost: the entries of the two lists in
// units of 8, at most 255); and the workgroup's histogram of the tile-order
// key (key[t], or the cost key when key is null), added into hist[256].
__global__ void __launch_bounds__(256) batch_caps_kernel(const uint2* __restrict__ ranges, ViewSet views, int batch,
                                                          const uint32_t* __restrict__ key, uint32_t* __restrict__ cost,
                                                          uint32_t* __restrict__ cur_off, uint32_t* __restrict__ blk,
                                                          uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[256];
    __shared__ uint32_t s_w[4];
    const int tid = threadIdx.x, lane = lane_id();
    h[tid] = 0u;
    __syncthreads();
    const uint32_t t = blockIdx.x * 256u + (uint32_t)tid;
    uint32_t c = 0;
    if (t < views.total_tiles) {
        int vi = 0;
        while (vi + 1 < views.n_views && t >= views.v[vi + 1].tile_off) ++vi;
        const DevView& cam = views.v[vi];
        const uint32_t lt = t - cam.tile_off;
        const int tx = (int)(lt % (uint32_t)cam.grid_w), ty = (int)(lt / (uint32_t)cam.grid_w);
        const uint2 r2 = ranges[region_of_tile(tx, ty, cam, views)];
        const uint32_t len1 = ranges[t].y - ranges[t].x;
        const uint32_t len2 = r2.y - r2.x;
        c = 2u * ((len1 + batch - 1) / batch + (len2 + batch - 1) / batch) + 2u;
        const uint32_t ck = min((len1 + len2) >> 3, 255u);
        if (cost) cost[t] = ck;
        atomicAdd(&h[255u - min(key ? key[t] : ck, 255u)], 1u);
    }
    uint32_t x = c;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    if (lane == 63) s_w[tid >> 6] = x;
    __syncthreads();
    uint32_t wo = 0;
    for (int v = 0; v < (tid >> 6); ++v) wo += s_w[v];
    if (t < views.total_tiles) cur_off[t] = wo + x - c;
    if (tid == 255) blk[blockIdx.x] = wo + x;
    if (h[tid]) atomicAdd(&hist[tid], h[tid]);
}

// Queue order of the tiles, most expensive first, so that the last tiles a
// persistent launch takes are cheap (its tail is the cost of the tiles
// still running when the queue runs dry).  A counting sort on a per-tile
// cost key (0..255, descending): order_hist_kernel adds every workgroup's
// histogram of the keys into hist[256]; order_place_kernel scans hist for the
// bins' starts, takes for each of its bins a run of slots with one atomic
// on cursor[256] and places its tiles in the run (ties in any order: the
// tiles are independent).  hist and cursor are zero before the first kernel.
__global__ void __launch_bounds__(256) order_hist_kernel(const uint32_t* __restrict__ key, uint32_t n,
                                                          uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[256];
    const int t = threadIdx.x;
    h[t] = 0u;
    __syncthreads();
    const uint32_t i = blockIdx.x * 256u + (uint32_t)t;
    if (i < n) atomicAdd(&h[255u - min(key[i], 255u)], 1u);
    __syncthreads();
    if (h[t]) atomicAdd(&hist[t], h[t]);
}

__global__ void __launch_bounds__(256) order_place_kernel(const uint32_t* __restrict__ key, uint32_t n,
                                                           const uint32_t* __restrict__ hist,
                                                           uint32_t* __restrict__ cursor, uint32_t* __restrict__ order) {
    __shared__ uint32_t s_base[256];
    __shared__ uint32_t s_cnt[256];
    __shared__ uint32_t s_wsum[4];
    const int t = threadIdx.x, lane = lane_id();
    // bin starts: exclusive scan of hist
    const uint32_t c = hist[t];
    uint32_t x = c;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    if (lane == 63) s_wsum[t >> 6] = x;
    s_cnt[t] = 0u;
    __syncthreads();
    uint32_t start = x - c;
    for (int v = 0; v < (t >> 6); ++v) start += s_wsum[v];
    // this workgroup's tiles per bin, and each tile's rank within its bin
    const uint32_t i = blockIdx.x * 256u + (uint32_t)t;
    const uint32_t b = i < n ? 255u - min(key[i], 255u) : 0u;
    const uint32_t rank = i < n ? atomicAdd(&s_cnt[b], 1u) : 0u;
    __syncthreads();
    // a run of slots per non-empty bin
    if (s_cnt[t]) s_base[t] = start + atomicAdd(&cursor[t], s_cnt[t]);
    __syncthreads();
    if (i < n) order[s_base[b] + rank] = i;
}

// order_place_kernel for the forward's set-up (the keys: key[t], or cost[t]
// when key is null), which also completes the checkpoint offsets: cur_off[t]
// (a prefix within its workgroup of 256 tiles) plus the totals of the
// earlier workgroups (blk), and *cur_need = the grand total.
__global__ void __launch_bounds__(256) order_offsets_kernel(const uint32_t* __restrict__ key,
                                                             const uint32_t* __restrict__ cost, uint32_t n,
                                                             const uint32_t* __restrict__ hist,
                                                             uint32_t* __restrict__ cursor,
                                                             uint32_t* __restrict__ order,
                                                             uint32_t* __restrict__ cur_off,
                                                             const uint32_t* __restrict__ blk,
                                                             uint64_t* __restrict__ cur_need) {
    __shared__ uint32_t s_base[256];
    __shared__ uint32_t s_cnt[256];
    __shared__ uint32_t s_wsum[4];
    __shared__ uint64_t s_pre[4];
    const int t = threadIdx.x, lane = lane_id();
    const uint32_t c = hist[t];
    uint32_t x = c;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    // checkpoints of the earlier workgroups
    uint64_t pre = 0;
    for (uint32_t b0 = 0; b0 < blockIdx.x; b0 += 256u) {
        const uint32_t b = b0 + (uint32_t)t;
        if (b < blockIdx.x) pre += blk[b];
    }
    for (int off = 32; off > 0; off >>= 1) pre += __shfl_xor(pre, off);
    if (lane == 63) s_wsum[t >> 6] = x;
    if (lane == 0) s_pre[t >> 6] = pre;
    s_cnt[t] = 0u;
    __syncthreads();
    uint32_t start = x - c;
    for (int v = 0; v < (t >> 6); ++v) start += s_wsum[v];
    const uint64_t before = s_pre[0] + s_pre[1] + s_pre[2] + s_pre[3];
    const uint32_t i = blockIdx.x * 256u + (uint32_t)t;
    if (i < n) cur_off[i] += (uint32_t)before;
    if (blockIdx.x == gridDim.x - 1 && t == 0) *cur_need = before + blk[blockIdx.x];
    const uint32_t b = i < n ? 255u - min(key ? key[i] : cost[i], 255u) : 0u;
    const uint32_t rank = i < n ? atomicAdd(&s_cnt[b], 1u) : 0u;
    __syncthreads();
    if (s_cnt[t]) s_base[t] = start + atomicAdd(&cursor[t], s_cnt[t]);
    __syncthreads();
    if (i < n) order[s_base[b] + rank] = i;
}

// ---------------------------------------------------------------------------
// merging two ordered streams in LDS
// ---------------------------------------------------------------------------

// Dynamic LDS of one workgroup for batch depth B: the staged records of the
// batch (3 float4 per entry) share their space with the merge windows, which
// are dead once the merged positions are known.
struct Lds {
    uint32_t* xk;     // narrow window (sorted positions)
    uint32_t* yraw;   // region window (sorted positions), before the tile test
    uint32_t* yk;     // entries of the region window that belong to this tile
    uint8_t* ypass;   // tile test of the region window
    // staged records of the batch, three float4 per entry (A, B, C): one
    // LDS address per entry, the three reads at fixed offsets
    float4* E;
    uint32_t* m;      // merged positions of the batch
    uint32_t* wsum;   // per-wave partial counts
};

__host__ __device__ constexpr size_t lds_bytes(int batch) { return (size_t)batch * (48 + 4) + 64; }

__device__ __forceinline__ Lds carve(char* smem, int batch) {
    Lds L;
    L.E = reinterpret_cast<float4*>(smem);
    L.xk = reinterpret_cast<uint32_t*>(smem);
    L.yraw = L.xk + batch;
    L.yk = L.yraw + batch;
    L.ypass = reinterpret_cast<uint8_t*>(L.yk + batch);
    L.m = reinterpret_cast<uint32_t*>(smem + 48 * (size_t)batch);
    L.wsum = L.m + batch;
    return L;
}

__device__ __forceinline__ int count_le(const uint32_t* a, int n, uint32_t key) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] <= key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int count_lt(const uint32_t* a, int n, uint32_t key) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Exclusive scan over a block of any multiple of 64 threads.
__device__ __forceinline__ uint32_t block_scan_excl(uint32_t v, uint32_t* wsum, uint32_t* total) {
    const int lane = lane_id(), w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (int i = 0; i < nw; ++i) {
        if (i < w) before += wsum[i];
        tot += wsum[i];
    }
    *total = tot;
    return before + x - v;
}

struct Batch {
    int M;      // staged entries (those that can reach a pixel of the tile)
    int Mfull;  // merged entries of the batch, staged or not
    int nX;     // narrow entries consumed
    int nYraw;  // region entries consumed (including those not belonging to the tile)
};

// Stages the next (at most `batch`) entries of the tile's merged list in LDS.
// Every thread of the block calls it; the result is uniform.  The first
// stream is the tile's narrow list, the second its region list, of which
// only the entries that reach the tile belong to the tile's list: with
// culling, those that pass the exact touch test (narrow lists are already
// culled the same way, so every merged entry is staged); without, those
// whose tile rectangle contains the tile (the list of Sec. 3.1), and the
// touch test then only decides which merged entries are staged.
__device__ Batch merge_batch(const Lds& L, const uint32_t* __restrict__ vals, const float4* __restrict__ srec,
                             int i1, int e1, int i2, int e2, int batch, int tcx, int tcy, const TileBox& tb,
                             const DevView& cam, const DevSettings& st, int kbase) {
    const int t = threadIdx.x, NT = blockDim.x;
    const int cX = min(batch, e1 - i1), cY = min(batch, e2 - i2);
    for (int l = t; l < cX; l += NT) L.xk[l] = vals[i1 + l];
    for (int l = t; l < cY; l += NT) {
        const uint32_t p = vals[i2 + l];
        L.yraw[l] = p;
        const float4 A = srec[3 * (size_t)p], B = srec[3 * (size_t)p + 1];
        bool pass;
        if (st.tile_cull) {
            pass = may_touch(A, B, tb, st);
        } else {
            const Rect q = rect_of(A.x, A.y, B.w, cam, st);
            pass = tcx >= q.x0 && tcx <= q.x1 && tcy >= q.y0 && tcy <= q.y1;
        }
        L.ypass[l] = pass ? 1 : 0;
    }
    __syncthreads();
    // entries up to the smaller of the two window ends are final (positions
    // are below 2^31, so the all-ones value means "no bound")
    uint32_t F = 0xffffffffu;
    if (i1 + cX < e1) F = L.xk[cX - 1];
    if (i2 + cY < e2) F = min(F, L.yraw[cY - 1]);
    int nX = count_le(L.xk, cX, F);
    int nYr = count_le(L.yraw, cY, F);
    // compact the passing entries among the consumed raw ones
    const int per = (cY + NT - 1) / NT;
    uint32_t cnt = 0;
    for (int q = 0; q < per; ++q) {
        const int l = t * per + q;
        if (l < nYr) cnt += L.ypass[l];
    }
    uint32_t nYu;
    uint32_t pos = block_scan_excl(cnt, L.wsum, &nYu);
    for (int q = 0; q < per; ++q) {
        const int l = t * per + q;
        if (l < nYr && L.ypass[l]) L.yk[pos++] = L.yraw[l];
    }
    __syncthreads();
    int nY = (int)nYu;
    if (nX + nY > batch) {
        // keep the `batch` smallest: co-rank of the diagonal d = batch
        const int d = batch;
        int lo = max(0, d - nY), hi = min(d, nX);
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (L.xk[mid] < L.yk[d - mid - 1]) lo = mid + 1;
            else hi = mid;
        }
        const int a = lo;
        uint32_t last = 0;
        if (a > 0) last = L.xk[a - 1];
        if (d - a > 0) last = max(last, L.yk[d - a - 1]);
        nX = a;
        nY = d - a;
        nYr = count_le(L.yraw, nYr, last);
    }
    for (int a = t; a < nX; a += NT) L.m[a + count_lt(L.yk, nY, L.xk[a])] = L.xk[a];
    for (int b = t; b < nY; b += NT) L.m[b + count_lt(L.xk, nX, L.yk[b])] = L.yk[b];
    __syncthreads();
    // the windows are dead: stage over them, in merged order, the records
    // that can reach a pixel of the tile (a and gamma scaled for
    // eval_entry); B.w (the radius, unused here) carries the entry's index
    // in the tile's full list: kbase (the merged entries of the earlier
    // batches) plus its index within the merged batch
    const int M = nX + nY;
    if (st.tile_cull) {
        for (int j = t; j < M; j += NT) {
            const size_t i = L.m[j];
            float4 B = stage_b(srec[3 * i + 1]);
            B.w = __int_as_float(kbase + j);
            L.E[3 * j] = stage_a(srec[3 * i]);
            L.E[3 * j + 1] = B;
            L.E[3 * j + 2] = srec[3 * i + 2];
        }
        __syncthreads();
        return Batch{M, M, nX, nYr};
    }
    const int run = (M + NT - 1) / NT;  // contiguous entries per thread (<= MAXB / 64)
    uint32_t keep = 0, nkeep = 0;
    for (int q = 0; q < run; ++q) {
        const int j = t * run + q;
        if (j < M) {
            const size_t i = L.m[j];
            if (may_touch(srec[3 * i], srec[3 * i + 1], tb, st)) {
                keep |= 1u << q;
                ++nkeep;
            }
        }
    }
    uint32_t Mc;
    uint32_t p = block_scan_excl(nkeep, L.wsum, &Mc);
    for (int q = 0; q < run; ++q) {
        if (!((keep >> q) & 1u)) continue;
        const int j = t * run + q;
        const size_t i = L.m[j];
        float4 B = stage_b(srec[3 * i + 1]);
        B.w = __int_as_float(kbase + j);
        L.E[3 * p] = stage_a(srec[3 * i]);
        L.E[3 * p + 1] = B;
        L.E[3 * p + 2] = srec[3 * i + 2];
        ++p;
    }
    __syncthreads();
    return Batch{(int)Mc, M, nX, nYr};
}

// Wave totals of ten per-lane quantities, each left in the lanes that
// issue its atomic.  The gfx950 lane swaps halve the data without selects:
// permlane32_swap trades the upper half of its first operand for the lower
// half of its second, so the sum of its two results holds the first
// quantity's total over lanes l, l + 32 in the lower half and the second's in
// the upper half; permlane16_swap trades rows 1 and 3 of its first operand
// for rows 0 and 2 of its second, which halves again across the row pairs.
// Four DPP steps within each 16-lane row then complete the totals.
__device__ __forceinline__ float dpp_xor1(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xb1, 0xf, 0xf, false));
}
__device__ __forceinline__ float dpp_xor2(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x4e, 0xf, 0xf, false));
}
__device__ __forceinline__ float dpp_ror4(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x124, 0xf, 0xf, false));
}
__device__ __forceinline__ float dpp_ror8(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x128, 0xf, 0xf, false));
}
__device__ __forceinline__ float halves_pair(float a, float b) {
    const auto s = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(s[0]) + __uint_as_float(s[1]);
}
__device__ __forceinline__ float rows_pair(float a, float b) {
    const auto s = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    return __uint_as_float(s[0]) + __uint_as_float(s[1]);
}
// total over the 16 lanes of each row, in every lane of the row
__device__ __forceinline__ float row_total(float x) {
    x += dpp_ror8(x);
    x += dpp_ror4(x);
    x += dpp_xor2(x);
    return x + dpp_xor1(x);
}

// Quantity whose wave total lane holds after wave_sum_swap10 (-1: none).
// Column 0 of the rows holds quantities 0, 2, 1, 3 (rows 0 to 3), column 1
// quantities 4, 6, 5, 7, column 2 of rows 0 and 2 quantities 8 and 9.
__device__ __forceinline__ int swap10_quantity(int lane) {
    const int row = lane >> 4, c = lane & 15;
    if (c == 0) return (row & 1) * 2 + (row >> 1);
    if (c == 1) return 4 + (row & 1) * 2 + (row >> 1);
    if (c == 2 && (row & 1) == 0) return 8 + (row >> 1);
    return -1;
}

__device__ __forceinline__ float wave_sum_swap10(const float (&v)[10], int lane) {
    const float s0 = halves_pair(v[0], v[1]), s1 = halves_pair(v[2], v[3]), s2 = halves_pair(v[4], v[5]);
    const float s3 = halves_pair(v[6], v[7]), s4 = halves_pair(v[8], v[9]);
    const float t0 = row_total(rows_pair(s0, s1));  // rows: quantities 0, 2, 1, 3
    const float t1 = row_total(rows_pair(s2, s3));  // rows: 4, 6, 5, 7
    const float t2 = row_total(rows_pair(s4, s4));  // rows: 8, 8, 9, 9
    const int c = lane & 15;
    return c == 0 ? t0 : (c == 1 ? t1 : t2);
}

// Pixel of slot i of thread t: every wave's slot covers one 8x8 block of
// the tile (block w PPT + i of the tile's TW / 8 x TH / 8 blocks), so that an
// entry whose footprint covers part of the tile leaves fewer lanes idle than
// with rows of the tile per slot.
template <int TW, int PPT>
__device__ __forceinline__ void pixel_of(int t, int i, const TileGeom& tg, int& x, int& y) {
    const int b = (t >> 6) * PPT + i, l = t & 63;
    x = tg.tx0 + (b % (TW / 8)) * 8 + (l & 7);
    y = tg.ty0 + (b / (TW / 8)) * 8 + (l >> 3);
}

// Staged-list chunks: a persistent workgroup composites many tiles, a plain
// one a single tile.
constexpr uint32_t STG_CHUNK_PERSISTENT = 4096;
constexpr uint32_t STG_CHUNK = 256;

struct HybridLists {
    const uint32_t* vals;      // list entries (sorted positions) in (cell, position) order
    const uint2* ranges;       // [start, end) per tile, then per region
    uint4* cur;                // batch checkpoints (narrow cursor, region cursor, merged index)
    const uint32_t* cur_off;   // first checkpoint of each tile
    uint32_t* nbatch;          // batches the forward took per tile
    const uint64_t* cur_need;  // checkpoints the tiles may take (device)
    uint64_t cur_cap;          // checkpoints the buffer holds
    uint32_t* flags;
    // entries the forward staged per batch, kept for the backward:
    // per checkpoint (offset into stg or all ones, count), and per staged
    // entry (sorted position, index within the merged batch)
    uint2* cur_stg;
    uint2* stg;                // null: the backward merges again
    uint32_t* stg_count;
    uint64_t stg_cap;
    double* drec_clear;        // the backward's FP64 accumulator, cleared by the forward
    uint64_t drec_clear_n2;    // its size in pairs of doubles
    const uint32_t* order;     // optional: tile taken at each queue position
};

// Both compositing kernels are built for at least five waves per SIMD (at
// most 96 registers), the forward with up to two pixels per thread for seven
// (72 registers): both spill a few values at most, and all run faster than
// with fewer waves (measured on the batched workload: forward 0.65 -> 0.63
// ms at four pixels per thread, 0.62 -> 0.58 ms at two; backward 1.02 ->
// 0.99 ms; eight waves for the forward spill more and are slower).
// STATS: write the per-pixel work counters (stats_out, eval_out).
// IMP: accumulate every Gaussian's blending weights M alpha T over the
// pixels it enters: the wave's sum (FP64 atomic) into imp_sum and its
// maximum (as float bits, the weights being non-negative) into imp_max.
template <int TW, int TH, int PPT, bool STATS, bool IMP>
__global__ void __launch_bounds__(TW * TH / PPT, PPT >= 4 ? 5 : 7) hybrid_fwd_kernel(
    const float4* __restrict__ srec, HybridLists hl, ViewSet views, DevSettings st, float* __restrict__ images,
    float* __restrict__ t_final, int32_t* __restrict__ last_out, int4* __restrict__ stats_out,
    int4* __restrict__ eval_out, uint32_t* __restrict__ queue, int64_t n, double* __restrict__ imp_sum,
    uint32_t* __restrict__ imp_max) {
    constexpr int NT = TW * TH / PPT;
    extern __shared__ __align__(16) char smem[];
    __shared__ uint32_t s_tile;
    const int t = threadIdx.x;
    const int batch = st.batch;
    const Lds L = carve(smem, batch);
    const EvalConsts ek = eval_consts(st);
    if (*hl.cur_need > hl.cur_cap) {  // a fixed workspace too small: report, write nothing
        if (blockIdx.x == 0 && t == 0) atomicOr(hl.flags, FLAG_CAPACITY);
        return;
    }
    // staged-list chunk of this workgroup (used by thread 0 only)
    const uint32_t chunk = queue ? STG_CHUNK_PERSISTENT : STG_CHUNK;
    uint32_t cbase = 0, cused = chunk;
    for (;;) {
        const uint32_t q = next_tile(queue, &s_tile, blockIdx.x);
        if (q >= views.total_tiles) break;
        const uint32_t tile = hl.order ? hl.order[q] : q;
        const TileGeom tg = tile_geom(views, tile, TW, TH);
        const DevView& cam = views.v[tg.vi];
        float px[PPT], py[PPT], T[PPT], C0[PPT], C1[PPT], C2[PPT];
        // stopk: the entry at which the pixel stopped, -1 while it runs
        // (and 0 for a pixel outside the view, which never runs): the
        // pixel's done flag, tested with one compare per slot and entry; its
        // value changes only when the pixel stops
        int last[PPT], stopk[PPT], nblend[PPT], nmasked[PPT], nev[PPT], nev_last[PPT];
        bool inside[PPT];
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            int x, y;
            pixel_of<TW, PPT>(t, i, tg, x, y);
            inside[i] = x < cam.width && y < cam.height;
            px[i] = (float)x + 0.5f;
            py[i] = (float)y + 0.5f;
            T[i] = 1.f;
            C0[i] = C1[i] = C2[i] = 0.f;
            last[i] = -1;
            stopk[i] = inside[i] ? -1 : 0;
            nblend[i] = nmasked[i] = nev[i] = nev_last[i] = 0;
        }
        const int tcx = tg.tx0 / TW, tcy = tg.ty0 / TH;
        const uint2 r1 = hl.ranges[tile];
        const uint2 r2 = hl.ranges[region_of_tile(tcx, tcy, cam, views)];
        const int e1 = (int)r1.y, e2 = (int)r2.y;
        int i1 = (int)r1.x, i2 = (int)r2.x, m = 0, b = 0;
        const TileBox tb{(float)tg.tx0 + 0.5f, (float)min(tg.tx0 + TW, cam.width) - 0.5f, (float)tg.ty0 + 0.5f,
                         (float)min(tg.ty0 + TH, cam.height) - 0.5f};
        uint4* cur = hl.cur + hl.cur_off[tile];
        while (i1 < e1 || i2 < e2) {
            bool active = false;
#pragma unroll
            for (int i = 0; i < PPT; ++i) active |= stopk[i] < 0;
            if (!__syncthreads_or(active)) break;
            if (t == 0) cur[b] = make_uint4((uint32_t)i1, (uint32_t)i2, (uint32_t)m, 0u);
            const Batch bt = merge_batch(L, hl.vals, srec, i1, e1, i2, e2, batch, tcx, tcy, tb, cam, st, m);
            // room for the staged entries in the list kept for the backward:
            // thread 0 sub-allocates from a chunk the workgroup took from the
            // global counter (one atomic per chunk, not per batch)
            uint32_t my_off = 0;
            if (hl.stg && t == 0) {
                if (cused + (uint32_t)bt.M > chunk) {
                    cbase = atomicAdd(hl.stg_count, chunk);
                    cused = 0;
                }
                my_off = cbase + cused;
                cused += (uint32_t)bt.M;
            }
            // uniform: a scalar loop bound
            const int Mb = __builtin_amdgcn_readfirstlane(bt.M);
            for (int j = 0; j < Mb; ++j) {
                // the wave leaves the batch once all its pixels are done,
                // tested every 16 entries (a done pixel's slot costs only
                // its skip; a test per entry costs more than it saves)
                if ((j & 15) == 0) {
                    active = false;
#pragma unroll
                    for (int i = 0; i < PPT; ++i) active |= stopk[i] < 0;
                    if (!__any(active)) break;
                }
                const float4 A = L.E[3 * j], B = L.E[3 * j + 1], Cc = L.E[3 * j + 2];
                const int k = __float_as_int(B.w);  // index in the tile's full list
                float isum = 0.f, imax = 0.f;
#pragma unroll
                for (int i = 0; i < PPT; ++i) {
                    if (stopk[i] >= 0) continue;
                    if (STATS) ++nev[i];
                    Eval e;
                    if (!eval_entry(A, B, px[i], py[i], ek, e)) continue;
                    const float ma = B.z * e.alpha;
                    const float test = T[i] * (1.f - ma);
                    // one select, not a branch with copies on both sides
                    const bool stop = test < st.t_min;
                    stopk[i] = stop ? k : stopk[i];
                    asm volatile("" : "+v"(stopk[i]));  // keeps the select here
                    if (stop) continue;
                    const float wgt = ma * T[i];
                    C0[i] += wgt * Cc.x;
                    C1[i] += wgt * Cc.y;
                    C2[i] += wgt * Cc.z;
                    T[i] = test;
                    last[i] = k;
                    if (STATS) {
                        ++nblend[i];
                        nmasked[i] += B.z == 0.f;
                        nev_last[i] = nev[i];
                    }
                    if (IMP) {
                        isum += wgt;
                        imax = fmaxf(imax, wgt);
                    }
                }
                if (IMP && __any(isum > 0.f)) {
                    const float ws = wave_sum(isum), wm = wave_max(imax);
                    if (lane_id() == 0) {
                        const int64_t g = (int64_t)__float_as_uint(Cc.w) - (int64_t)tg.vi * n;
                        atomicAdd(imp_sum + g, (double)ws);
                        atomicMax(imp_max + g, __float_as_uint(wm));
                    }
                }
            }
            active = false;
#pragma unroll
            for (int i = 0; i < PPT; ++i) active |= stopk[i] < 0;
            if (hl.stg) {
                if (t == 0) {
                    const uint32_t off = (uint64_t)my_off + (uint64_t)bt.M <= hl.stg_cap ? my_off : 0xffffffffu;
                    L.wsum[8] = off;
                    hl.cur_stg[hl.cur_off[tile] + b] = make_uint2(off, (uint32_t)bt.M);
                }
                __syncthreads();
                const uint32_t off = L.wsum[8];
                if (off != 0xffffffffu) {
                    for (int p = t; p < bt.M; p += NT) {
                        const uint32_t jj = __float_as_uint(L.E[3 * p + 1].w) - (uint32_t)m;
                        hl.stg[off + p] = make_uint2(L.m[jj], jj);
                    }
                }
            }
            i1 += bt.nX;
            i2 += bt.nYraw;
            m += bt.Mfull;
            ++b;
            __syncthreads();  // the next batch overwrites the LDS
        }
        if (t == 0) hl.nbatch[tile] = (uint32_t)b;
        if (hl.drec_clear) {
            // the backward's FP64 accumulator of per-record gradients is
            // cleared here, one slice per tile: this kernel is bound by VALU
            // issue and leaves HBM bandwidth idle, the projection backward
            // (HBM-bound) then only reads the rows
            const uint64_t per = (hl.drec_clear_n2 + views.total_tiles - 1) / views.total_tiles;
            const uint64_t q0 = (uint64_t)tile * per;
            const uint64_t q1 = min(q0 + per, hl.drec_clear_n2);
            double2* z = reinterpret_cast<double2*>(hl.drec_clear);
            for (uint64_t q = q0 + (uint64_t)t; q < q1; q += NT) z[q] = make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            if (!inside[i]) continue;
            int x, y;
            pixel_of<TW, PPT>(t, i, tg, x, y);
            const int64_t pv = (int64_t)cam.width * cam.height;
            const int64_t loc = (int64_t)y * cam.width + x;
            float* im = images + 3 * (int64_t)cam.px_off;
            im[loc] = C0[i] + T[i] * st.bg[0];
            im[pv + loc] = C1[i] + T[i] * st.bg[1];
            im[2 * pv + loc] = C2[i] + T[i] * st.bg[2];
            const int64_t p = (int64_t)cam.px_off + loc;
            t_final[p] = T[i];
            last_out[p] = last[i];
            // a pixel that never stopped saw the whole merged list (m entries);
            // entries it evaluated are those of the list that can reach the tile
            if (STATS) {
                stats_out[p] = make_int4(stopk[i] >= 0 ? stopk[i] + 1 : m, nblend[i], nmasked[i], last[i] + 1);
                eval_out[p] = make_int4(nev[i], nev_last[i], 0, 0);
            }
        }
        if (!queue) break;
    }
}

template <int TW, int TH, int PPT>
__global__ void __launch_bounds__(TW * TH / PPT, 5) hybrid_bwd_kernel(
    const float4* __restrict__ srec, HybridLists hl, ViewSet views, DevSettings st, const float* __restrict__ t_final,
    const int32_t* __restrict__ last_in, const float* __restrict__ dl_dimages, int64_t n, double* __restrict__ d_rec,
    double* __restrict__ d_masks, uint32_t* __restrict__ queue) {
    constexpr int NT = TW * TH / PPT;
    extern __shared__ __align__(16) char smem[];
    __shared__ uint32_t s_tile;
    __shared__ int s_top;
    const int t = threadIdx.x;
    const int lane = lane_id();
    const int batch = st.batch;
    const Lds L = carve(smem, batch);
    const float bg0 = st.bg[0], bg1 = st.bg[1], bg2 = st.bg[2];
    const EvalConsts ek = eval_consts(st);
    // the quantity whose wave total this lane adds into the accumulator
    // (-1: none); the totals of the sums over t^2 and dy^2 (quantities 2
    // and 4) are rescaled by QSCALE / 2 to give dL/da and dL/dgamma (see the
    // pixel loop)
    const int qi = swap10_quantity(lane);
    const float qscale = (qi == 2 || qi == 4) ? 0.5f * QSCALE : 1.f;
    if (*hl.cur_need > hl.cur_cap) return;  // the forward reported it
    for (;;) {
        const uint32_t q = next_tile(queue, &s_tile, blockIdx.x);
        if (q >= views.total_tiles) break;
        const uint32_t tile = hl.order ? hl.order[q] : q;
        const TileGeom tg = tile_geom(views, tile, TW, TH);
        const DevView& cam = views.v[tg.vi];
        const int64_t rec_base = (int64_t)tg.vi * n;
        // s = w . b: the loss weights of the pixel dotted with the colour
        // composited behind the current entry (scaled by its transmittance)
        float px[PPT], py[PPT], T[PPT], Tf[PPT], w0[PPT], w1[PPT], w2[PPT], wbg[PPT], sb[PPT];
        int lastk[PPT];
        int mylast = -1;
        const int64_t pv = (int64_t)cam.width * cam.height;
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            int x, y;
            pixel_of<TW, PPT>(t, i, tg, x, y);
            px[i] = (float)x + 0.5f;
            py[i] = (float)y + 0.5f;
            sb[i] = 0.f;
            if (x < cam.width && y < cam.height) {
                const int64_t loc = (int64_t)y * cam.width + x;
                const int64_t p = (int64_t)cam.px_off + loc;
                const float* dl = dl_dimages + 3 * (int64_t)cam.px_off;
                lastk[i] = last_in[p];
                Tf[i] = t_final[p];
                w0[i] = dl[loc];
                w1[i] = dl[pv + loc];
                w2[i] = dl[2 * pv + loc];
            } else {
                lastk[i] = -1;
                Tf[i] = 1.f;
                w0[i] = w1[i] = w2[i] = 0.f;
            }
            T[i] = Tf[i];
            wbg[i] = w0[i] * bg0 + w1[i] * bg1 + w2[i] * bg2;
            mylast = max(mylast, lastk[i]);
        }
        for (int off = 32; off > 0; off >>= 1) mylast = max(mylast, __shfl_xor(mylast, off));
        if (t == 0) s_top = -1;
        __syncthreads();
        if (lane == 0) atomicMax(&s_top, mylast);
        __syncthreads();
        const int top = s_top;
        const uint4* cur = hl.cur + hl.cur_off[tile];
        const int tcx = tg.tx0 / TW, tcy = tg.ty0 / TH;
        const uint2 r1 = hl.ranges[tile];
        const uint2 r2 = hl.ranges[region_of_tile(tcx, tcy, cam, views)];
        const TileBox tb{(float)tg.tx0 + 0.5f, (float)min(tg.tx0 + TW, cam.width) - 0.5f, (float)tg.ty0 + 0.5f,
                         (float)min(tg.ty0 + TH, cam.height) - 0.5f};
        // the batch holding the largest last-blended entry, then backwards
        int bstar = -1;
        if (top >= 0) {
            const int nb = (int)hl.nbatch[tile];
            for (int b = 0; b < nb; ++b)
                if ((int)cur[b].z <= top) bstar = b;
        }
        const uint2* cstg = hl.stg ? hl.cur_stg + hl.cur_off[tile] : nullptr;
        // per-entry partial sums of this lane's pixels; zero between entries
        // (reset after each reduction), so no per-entry initialisation
        float gu = 0.f, gv = 0.f, ga = 0.f, gb = 0.f, gc = 0.f, go = 0.f, gr = 0.f, gg = 0.f, gbl = 0.f, gm = 0.f;
        for (int b = bstar; b >= 0; --b) {
            const uint4 c = cur[b];
            const int m = (int)c.z;
            const uint2 cs = cstg ? cstg[b] : make_uint2(0xffffffffu, 0u);
            int Mb;
            if (cs.x != 0xffffffffu) {
                // the entries the forward staged for this batch
                Mb = (int)cs.y;
                for (int p = t; p < Mb; p += NT) {
                    const uint2 e = hl.stg[cs.x + p];
                    const size_t i = e.x;
                    float4 B = stage_b(srec[3 * i + 1]);
                    B.w = __int_as_float(m + (int)e.y);
                    L.E[3 * p] = stage_a(srec[3 * i]);
                    L.E[3 * p + 1] = B;
                    L.E[3 * p + 2] = srec[3 * i + 2];
                }
                __syncthreads();
            } else {
                Mb = merge_batch(L, hl.vals, srec, (int)c.x, (int)r1.y, (int)c.y, (int)r2.y, batch, tcx, tcy, tb,
                                 cam, st, m).M;
            }
            for (int j = Mb - 1; j >= 0; --j) {
                const float4 A = L.E[3 * j], B = L.E[3 * j + 1], Cc = L.E[3 * j + 2];
                const int k = __float_as_int(B.w);  // index in the tile's full list
                if (k > top) continue;                  // uniform: past every pixel's last entry
                const float M = B.z;
                const float okq = B.y * QSCALE_NINV;
                bool any = false;
#pragma unroll
                for (int i = 0; i < PPT; ++i) {
                    if (k > lastk[i]) continue;
                    Eval e;
                    if (!eval_entry(A, B, px[i], py[i], ek, e)) continue;
                    any = true;
                    const float ma = M * e.alpha;
                    const float one_m = 1.f - ma;
                    const float inv = __builtin_amdgcn_rcpf(one_m);
                    const float Ti = T[i] * inv;
                    const float d = fmaf(w0[i], Cc.x, fmaf(w1[i], Cc.y, w2[i] * Cc.z)) - sb[i];
                    const float X = Ti * d - Tf[i] * inv * wbg[i];
                    gm += e.alpha * X;
                    const float wt = ma * Ti;
                    gr += wt * w0[i];
                    gg += wt * w1[i];
                    gbl += wt * w2[i];
                    if (e.oG <= ek.amax) {
                        // dL/dalpha = M X, dL/dQ = -o G M X / 2; with a' = QSCALE a,
                        // gamma' = QSCALE gamma: dL/du = kq a' t, dL/dv =
                        // kq (beta a' t + gamma' dy), dL/dbeta = kq a' t dy, and
                        // dL/da, dL/dgamma are QSCALE / 2 times the sums of kq t^2,
                        // kq dy^2, where kq = 2 dL/dQ / QSCALE
                        const float GdA = e.G * (M * X);
                        go += GdA;
                        const float kq = GdA * okq;
                        const float kapt = kq * e.apt;
                        gu += kapt;
                        gv += kq * fmaf(A.w, e.apt, e.gdy);
                        gb += kapt * e.dy;
                        ga += (kq * e.t) * e.t;
                        gc += (kq * e.dy) * e.dy;
                    }
                    sb[i] = fmaf(ma, d, sb[i]);
                    T[i] = Ti;
                }
                if (__any(any)) {
                    const uint32_t r = __float_as_uint(Cc.w);
                    const int64_t g = (int64_t)r - rec_base;
                    if (M != 0.f) {
                        // ten lanes receive the wave totals, quantity qi each
                        const float v[10] = {gu, gv, ga, gb, gc, go, gr, gg, gbl, gm};
                        const float x = wave_sum_swap10(v, lane) * qscale;
                        if ((unsigned)qi < (unsigned)DREC) atomicAdd(d_rec + (size_t)r * DREC + qi, (double)x);
                        else if (qi == DREC) atomicAdd(d_masks + g, (double)x);
                    } else {
                        const float sm = wave_sum(gm);
                        if (lane == 0) atomicAdd(d_masks + g, (double)sm);
                    }
                    gu = gv = ga = gb = gc = go = gr = gg = gbl = gm = 0.f;
                }
            }
            __syncthreads();  // the next batch overwrites the LDS
        }
        if (!queue) break;
    }
}

// Persistent grid per batch depth (index log2(batch / 32)).
template <typename Kernel>
int cached_grid(int (&cache)[4], Kernel k, int block, int num_cus, int batch) {
    const int idx = batch <= 32 ? 0 : batch <= 64 ? 1 : batch <= 128 ? 2 : 3;
    if (!cache[idx]) cache[idx] = persistent_grid(k, block, num_cus, lds_bytes(batch));
    return cache[idx];
}

template <int TW, int TH, int PPT, bool STATS, bool IMP>
void hybrid_fwd_s(hipStream_t s, int num_cus, const float* srec, const HybridLists& hl, const ViewSet& views,
                  const DevSettings& st, float* images, float* t_final, int32_t* last, int32_t* stats,
                  int32_t* evals, uint32_t* queue, int64_t n, double* imp_sum, uint32_t* imp_max) {
    int grid = (int)views.total_tiles;
    if (queue) {
        static int cache[4] = {0, 0, 0, 0};
        grid = min(cached_grid(cache, hybrid_fwd_kernel<TW, TH, PPT, STATS, IMP>, TW * TH / PPT, num_cus,
                               st.batch),
                   grid);
    }
    hipLaunchKernelGGL((hybrid_fwd_kernel<TW, TH, PPT, STATS, IMP>), dim3(grid), dim3(TW * TH / PPT),
                       lds_bytes(st.batch), s, reinterpret_cast<const float4*>(srec), hl, views, st, images, t_final,
                       last, reinterpret_cast<int4*>(stats), reinterpret_cast<int4*>(evals), queue, n, imp_sum,
                       imp_max);
}

template <int TW, int TH, int PPT>
void hybrid_fwd_t(hipStream_t s, int num_cus, const float* srec, const HybridLists& hl, const ViewSet& views,
                  const DevSettings& st, float* images, float* t_final, int32_t* last, int32_t* stats,
                  int32_t* evals, uint32_t* queue, int64_t n, double* imp_sum, uint32_t* imp_max) {
    if (imp_sum && imp_max)
        hybrid_fwd_s<TW, TH, PPT, false, true>(s, num_cus, srec, hl, views, st, images, t_final, last, nullptr,
                                               nullptr, queue, n, imp_sum, imp_max);
    else if (stats && evals)
        hybrid_fwd_s<TW, TH, PPT, true, false>(s, num_cus, srec, hl, views, st, images, t_final, last, stats, evals,
                                               queue, n, nullptr, nullptr);
    else
        hybrid_fwd_s<TW, TH, PPT, false, false>(s, num_cus, srec, hl, views, st, images, t_final, last, nullptr,
                                                nullptr, queue, n, nullptr, nullptr);
}

template <int TW, int TH, int PPT>
void hybrid_bwd_t(hipStream_t s, int num_cus, const float* srec, const HybridLists& hl, const ViewSet& views,
                  const DevSettings& st, const float* t_final, const int32_t* last, const float* dl, int64_t n,
                  double* d_rec, double* d_masks, uint32_t* queue) {
    int grid = (int)views.total_tiles;
    if (queue) {
        static int cache[4] = {0, 0, 0, 0};
        grid = min(cached_grid(cache, hybrid_bwd_kernel<TW, TH, PPT>, TW * TH / PPT, num_cus, st.batch), grid);
    }
    hipLaunchKernelGGL((hybrid_bwd_kernel<TW, TH, PPT>), dim3(grid), dim3(TW * TH / PPT), lds_bytes(st.batch), s,
                       reinterpret_cast<const float4*>(srec), hl, views, st, t_final, last, dl, n, d_rec, d_masks,
                       queue);
}

#define MGS_HYBRID_SHAPES(X) \
    X(8, 8, 1)               \
    X(16, 8, 1)              \
    X(16, 8, 2)              \
    X(16, 16, 1)             \
    X(16, 16, 2)             \
    X(16, 16, 4)             \
    X(32, 8, 1)              \
    X(32, 8, 2)              \
    X(32, 8, 4)

HybridLists make_lists(const HybridBuffers& b) {
    HybridLists hl;
    hl.vals = b.vals;
    hl.ranges = reinterpret_cast<const uint2*>(b.ranges);
    hl.cur = reinterpret_cast<uint4*>(b.cur);
    hl.cur_off = b.cur_off;
    hl.nbatch = b.nbatch;
    hl.cur_need = b.cur_need;
    hl.cur_cap = b.cur_cap;
    hl.flags = b.flags;
    hl.cur_stg = reinterpret_cast<uint2*>(b.cur_stg);
    hl.stg = reinterpret_cast<uint2*>(b.stg);
    hl.stg_count = b.stg_count;
    hl.order = b.order;
    hl.stg_cap = b.stg_cap;
    hl.drec_clear = b.drec_clear;
    hl.drec_clear_n2 = b.drec_clear_n2;
    return hl;
}

unsigned blocks_of(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

bool composite_config_supported(const CompositeConfig& c) {
#define MGS_MATCH(A, B, P) \
    if (c.tile_w == A && c.tile_h == B && c.ppt == P) return true;
    MGS_HYBRID_SHAPES(MGS_MATCH)
#undef MGS_MATCH
    return false;
}

void launch_permute_classify(hipStream_t stream, const uint32_t* order, const uint32_t* skeys, const float* rec,
                             int64_t R, int64_t n, const ViewSet& views, const DevSettings& st, uint32_t* cnt,
                             uint64_t* tmask, float* srec, uint32_t* part) {
    if (R == 0) return;
    const unsigned nb = blocks_of(R);
    hipLaunchKernelGGL(permute_classify_kernel, dim3(nb), dim3(256), 0, stream, order, skeys,
                       reinterpret_cast<const float4*>(rec), R, n, views, st, cnt, tmask,
                       reinterpret_cast<float4*>(srec), part);
}

// part: 2 nb + 4 nb u32 counts (per workgroup, per wave), then (8-byte
// aligned) the list offsets: per wave, per group (3 totals and the offset)
namespace {
int64_t waves_of(int64_t R) { return (int64_t)blocks_of(R) * 4; }
int64_t groups_of(int64_t R) { return (waves_of(R) + LO_GROUP - 1) / LO_GROUP; }
size_t counts_bytes(int64_t R) { return ((size_t)blocks_of(R) * 24 + 15) / 8 * 8; }
ListOffsets list_offsets(uint32_t* part, int64_t R) {
    char* p = reinterpret_cast<char*>(part) + counts_bytes(R);
    ListOffsets lo;
    lo.wave_rel = reinterpret_cast<uint64_t*>(p);
    lo.group_tot = lo.wave_rel + waves_of(R);
    lo.group_off = lo.group_tot + 3 * groups_of(R);
    return lo;
}
}  // namespace

size_t classify_parts_bytes(int64_t R) { return counts_bytes(R) + (size_t)(waves_of(R) + 4 * groups_of(R)) * 8 + 8; }

void launch_list_offsets(hipStream_t stream, uint32_t* part, int64_t R, uint64_t* total, uint64_t* wide_counts) {
    const ListOffsets lo = list_offsets(part, R);
    const int64_t ng = R > 0 ? groups_of(R) : 0;
    if (ng > 0)
        hipLaunchKernelGGL(list_offsets_group_kernel, dim3((unsigned)ng), dim3(LO_GROUP), 0, stream, part,
                           (int64_t)blocks_of(R), waves_of(R), lo);
    hipLaunchKernelGGL(list_offsets_total_kernel, dim3(1), dim3(LO_GROUP), 0, stream, ng, lo, total, wide_counts);
}

void launch_duplicate_lists(hipStream_t stream, const float* srec, const uint32_t* cnt_sorted,
                            const uint64_t* tmask, uint32_t* part, int64_t R,
                            int64_t n, const ViewSet& views, const DevSettings& st, uint32_t* keys, uint32_t* vals,
                            int64_t capacity, uint32_t* flags) {
    if (R == 0) return;
    hipLaunchKernelGGL(duplicate_kernel, dim3(blocks_of(R)), dim3(256), 0, stream,
                       reinterpret_cast<const float4*>(srec), cnt_sorted, tmask, list_offsets(part, R), R,
                       n, views, st, keys, vals, capacity, flags);
}

void launch_tile_order(hipStream_t stream, const uint32_t* key, uint32_t tiles, uint32_t* hist_cursor,
                       uint32_t* order, bool cleared) {
    if (tiles == 0) return;
    if (!cleared) launch_fill_u32(stream, hist_cursor, 512, 0u);
    hipLaunchKernelGGL(order_hist_kernel, dim3(blocks_of(tiles)), dim3(256), 0, stream, key, tiles, hist_cursor);
    hipLaunchKernelGGL(order_place_kernel, dim3(blocks_of(tiles)), dim3(256), 0, stream, key, tiles,
                       (const uint32_t*)hist_cursor, hist_cursor + 256, order);
}

void launch_tile_setup(hipStream_t stream, const uint32_t* ranges, const ViewSet& views, int batch,
                       const uint32_t* key, uint32_t* cost, uint32_t* cur_off, uint64_t* cur_need, uint32_t* blk,
                       uint32_t* hist_cursor, uint32_t* order) {
    const uint32_t T = views.total_tiles;
    if (T == 0) return;
    hipLaunchKernelGGL(batch_caps_kernel, dim3(blocks_of(T)), dim3(256), 0, stream,
                       reinterpret_cast<const uint2*>(ranges), views, batch, key, cost, cur_off, blk, hist_cursor);
    hipLaunchKernelGGL(order_offsets_kernel, dim3(blocks_of(T)), dim3(256), 0, stream, key, (const uint32_t*)cost, T,
                       (const uint32_t*)hist_cursor, hist_cursor + 256, order, cur_off, (const uint32_t*)blk,
                       cur_need);
}

void launch_hybrid_fwd(hipStream_t stream, const CompositeConfig& cfg, const float* srec, const HybridBuffers& bufs,
                       const ViewSet& views, const DevSettings& st, float* images, float* t_final, int32_t* last,
                       int32_t* stats, int32_t* evals, uint32_t* queue, int num_cus, int64_t n, double* imp_sum,
                       uint32_t* imp_max) {
    if (views.total_tiles == 0) return;
    const HybridLists hl = make_lists(bufs);
#define MGS_HFWD(A, B, P)                                                                                          \
    if (cfg.tile_w == A && cfg.tile_h == B && cfg.ppt == P) {                                                      \
        hybrid_fwd_t<A, B, P>(stream, num_cus, srec, hl, views, st, images, t_final, last, stats, evals, queue, n, \
                              imp_sum, imp_max);                                                                   \
        return;                                                                                                    \
    }
    MGS_HYBRID_SHAPES(MGS_HFWD)
#undef MGS_HFWD
}

void launch_hybrid_bwd(hipStream_t stream, const CompositeConfig& cfg, const float* srec, const HybridBuffers& bufs,
                       const ViewSet& views, const DevSettings& st, const float* t_final, const int32_t* last,
                       const float* dl_dimages, int64_t n, double* d_rec, double* d_masks, uint32_t* queue,
                       int num_cus) {
    if (views.total_tiles == 0) return;
    const HybridLists hl = make_lists(bufs);
#define MGS_HBWD(A, B, P)                                                                                       \
    if (cfg.tile_w == A && cfg.tile_h == B && cfg.ppt == P) {                                                   \
        hybrid_bwd_t<A, B, P>(stream, num_cus, srec, hl, views, st, t_final, last, dl_dimages, n, d_rec, d_masks, \
                              queue);                                                                           \
        return;                                                                                                 \
    }
    MGS_HYBRID_SHAPES(MGS_HBWD)
#undef MGS_HBWD
}

}  // namespace mgs
