// Masked compositing on gfx950, forward and backward.
//
// Forward, per pixel and front to back over its tile's depth-sorted entries
// (Eq. 3-4): entries outside the 3-sigma cut or below the alpha filter are
// skipped; an entry that would take the transmittance below T_min stops the
// pixel and is excluded; otherwise C += M a T c and T *= (1 - M a).  The
// background adds T_final * bg (supplementary derivation).
//
// Backward, per pixel in reverse from its last blended entry: the
// transmittance in front of entry i is recovered by division,
// T_i = T_{i+1} / (1 - M_i a_i), and the colour behind is accumulated
// relative to T_{i+1} (b_i = M a c + (1 - M a) b_{i+1}).  With
//   X_i = T_i <w, c_i - b_{i+1}> - T_final / (1 - M_i a_i) <w, bg>,
// dL/dM_i = a_i X_i for every entry that passed the alpha filter whatever
// its mask (Eq. 6 and the background term), dL/da_i = M_i X_i and
// dL/dc_i = M_i a_i T_i w, so masked entries get only the mask gradient
// (Fig. 1).
//
// A workgroup owns one tile (tile_w x tile_h pixels); each thread owns PPT
// pixels, so a wave covers up to 256 pixels and the per-entry wave reduction
// of the backward is amortised over PPT pixels per lane.  Entries are staged
// through LDS in batches; a pixel leaves when it stops, a wave skips the rest
// of a batch when all its pixels have stopped, and the workgroup leaves the
// tile when every pixel has.  With a queue pointer the launch is persistent:
// workgroups pop tile ids from a device counter until the tiles run out.
#include "common.hpp"
#include "composite_common.hpp"
#include "kernels.hpp"

namespace mgs {
namespace {

template <int TW, int TH, int PPT>
__global__ void __launch_bounds__(TW * TH / PPT) composite_fwd_kernel(
    const float4* __restrict__ rec, const uint32_t* __restrict__ vals, const uint2* __restrict__ ranges,
    ViewSet views, DevSettings st, float* __restrict__ images, float* __restrict__ t_final,
    int32_t* __restrict__ last_out, int32_t* __restrict__ examined_out, int4* __restrict__ stats_out,
    uint32_t* __restrict__ queue) {
    constexpr int NT = TW * TH / PPT;
    __shared__ float4 sA[MAXB], sB[MAXB], sC[MAXB];
    __shared__ uint32_t s_tile;
    const int t = threadIdx.x;
    const int batch = st.batch;
    const EvalConsts ek = eval_consts(st);
    for (;;) {
        const uint32_t tile = next_tile(queue, &s_tile, blockIdx.x);
        if (tile >= views.total_tiles) break;
        const TileGeom tg = tile_geom(views, tile, TW, TH);
        const DevView& cam = views.v[tg.vi];
        float px[PPT], py[PPT], T[PPT], C0[PPT], C1[PPT], C2[PPT];
        int last[PPT], stopk[PPT], nblend[PPT], nmasked[PPT];
        bool done[PPT], inside[PPT];
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            const int pidx = t + i * NT;
            const int x = tg.tx0 + pidx % TW, y = tg.ty0 + pidx / TW;
            inside[i] = x < cam.width && y < cam.height;
            px[i] = (float)x + 0.5f;
            py[i] = (float)y + 0.5f;
            T[i] = 1.f;
            C0[i] = C1[i] = C2[i] = 0.f;
            last[i] = -1;
            stopk[i] = -1;
            nblend[i] = nmasked[i] = 0;
            done[i] = !inside[i];
        }
        const uint2 rg = ranges[tile];
        const int start = (int)rg.x, end = (int)rg.y;
        for (int base = start; base < end; base += batch) {
            bool active = false;
#pragma unroll
            for (int i = 0; i < PPT; ++i) active |= !done[i];
            if (!__syncthreads_or(active)) break;
            for (int l = t; l < batch; l += NT) {
                const int k = base + l;
                if (k < end) {
                    const uint32_t r = vals[k];
                    sA[l] = stage_a(rec[3 * (size_t)r]);
                    sB[l] = stage_b(rec[3 * (size_t)r + 1]);
                    sC[l] = rec[3 * (size_t)r + 2];
                }
            }
            __syncthreads();
            const int cnt = min(batch, end - base);
            for (int j = 0; j < cnt; ++j) {
                if (!__any(active)) break;
                const float4 A = sA[j], B = sB[j], Cc = sC[j];
#pragma unroll
                for (int i = 0; i < PPT; ++i) {
                    if (done[i]) continue;
                    Eval e;
                    if (!eval_entry(A, B, px[i], py[i], ek, e)) continue;
                    const float ma = B.z * e.alpha;
                    const float test = T[i] * (1.f - ma);
                    if (test < st.t_min) {
                        done[i] = true;
                        stopk[i] = base + j;
                        continue;
                    }
                    const float wgt = ma * T[i];
                    C0[i] += wgt * Cc.x;
                    C1[i] += wgt * Cc.y;
                    C2[i] += wgt * Cc.z;
                    T[i] = test;
                    last[i] = base + j;
                    ++nblend[i];
                    nmasked[i] += B.z == 0.f;
                }
                active = false;
#pragma unroll
                for (int i = 0; i < PPT; ++i) active |= !done[i];
            }
        }
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            if (!inside[i]) continue;
            const int pidx = t + i * NT;
            const int x = tg.tx0 + pidx % TW, y = tg.ty0 + pidx / TW;
            const int64_t pv = (int64_t)cam.width * cam.height;
            const int64_t loc = (int64_t)y * cam.width + x;
            float* im = images + 3 * (int64_t)cam.px_off;
            im[loc] = C0[i] + T[i] * st.bg[0];
            im[pv + loc] = C1[i] + T[i] * st.bg[1];
            im[2 * pv + loc] = C2[i] + T[i] * st.bg[2];
            const int64_t p = (int64_t)cam.px_off + loc;
            if (t_final) t_final[p] = T[i];
            if (last_out) last_out[p] = last[i];
            const int exam = stopk[i] >= 0 ? stopk[i] - start + 1 : end - start;
            if (examined_out) examined_out[p] = exam;
            if (stats_out) stats_out[p] = make_int4(exam, nblend[i], nmasked[i], last[i] >= 0 ? last[i] - start + 1 : 0);
        }
        if (!queue) break;
    }
}

template <int TW, int TH, int PPT>
__global__ void __launch_bounds__(TW * TH / PPT) composite_bwd_kernel(
    const float4* __restrict__ rec, const uint32_t* __restrict__ vals, const uint2* __restrict__ ranges,
    ViewSet views, DevSettings st, const float* __restrict__ t_final, const int32_t* __restrict__ last_in,
    const float* __restrict__ dl_dimages, int64_t n, float* __restrict__ d_rec, float* __restrict__ d_masks,
    uint32_t* __restrict__ queue) {
    constexpr int NT = TW * TH / PPT;
    __shared__ float4 sA[MAXB], sB[MAXB], sC[MAXB];
    __shared__ uint32_t sR[MAXB];
    __shared__ uint32_t s_tile;
    __shared__ int s_top;
    const int t = threadIdx.x;
    const int lane = lane_id();
    const int batch = st.batch;
    const float bg0 = st.bg[0], bg1 = st.bg[1], bg2 = st.bg[2];
    const EvalConsts ek = eval_consts(st);
    for (;;) {
        const uint32_t tile = next_tile(queue, &s_tile, blockIdx.x);
        if (tile >= views.total_tiles) break;
        const TileGeom tg = tile_geom(views, tile, TW, TH);
        const DevView& cam = views.v[tg.vi];
        const int64_t rec_base = (int64_t)tg.vi * n;
        // sb = w . b: the pixel's loss weights dotted with the colour composited
        // behind the current entry
        float px[PPT], py[PPT], T[PPT], Tf[PPT], w0[PPT], w1[PPT], w2[PPT], wbg[PPT], sb[PPT];
        int lastk[PPT];
        int mylast = -1;
        const int64_t pv = (int64_t)cam.width * cam.height;
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            const int pidx = t + i * NT;
            const int x = tg.tx0 + pidx % TW, y = tg.ty0 + pidx / TW;
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
        // the workgroup starts from the largest last-blended position
        for (int off = 32; off > 0; off >>= 1) mylast = max(mylast, __shfl_xor(mylast, off));
        if (t == 0) s_top = -1;
        __syncthreads();
        if (lane == 0) atomicMax(&s_top, mylast);
        __syncthreads();
        const int top0 = s_top;
        const int start = (int)ranges[tile].x;
        for (int top = top0; top >= start; top -= batch) {
            const int lo = max(start, top - batch + 1);
            const int cnt = top - lo + 1;
            __syncthreads();
            for (int l = t; l < cnt; l += NT) {
                const uint32_t r = vals[lo + l];
                sR[l] = r;
                sA[l] = stage_a(rec[3 * (size_t)r]);
                sB[l] = stage_b(rec[3 * (size_t)r + 1]);
                sC[l] = rec[3 * (size_t)r + 2];
            }
            __syncthreads();
            for (int j = cnt - 1; j >= 0; --j) {
                const int k = lo + j;
                const float4 A = sA[j], B = sB[j], Cc = sC[j];
                const float M = B.z;
                const float okq = B.y * QSCALE_NINV;
                float gu = 0.f, gv = 0.f, ga = 0.f, gb = 0.f, gc = 0.f, go = 0.f, gr = 0.f, gg = 0.f, gbl = 0.f,
                      gm = 0.f;
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
                        // conic terms as multiples of kq = 2 dL/dQ / QSCALE (the
                        // sums over t^2 and dy^2 are rescaled by QSCALE / 2 below)
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
                    const uint32_t r = sR[j];
                    const int64_t g = (int64_t)r - rec_base;
                    const float sm = wave_sum(gm);
                    if (M != 0.f) {
                        const float su = wave_sum(gu), sv = wave_sum(gv), sa = wave_sum(ga) * (0.5f * QSCALE),
                                    sbt = wave_sum(gb), sc = wave_sum(gc) * (0.5f * QSCALE), so = wave_sum(go),
                                    sr = wave_sum(gr), sg = wave_sum(gg), sbl = wave_sum(gbl);
                        float v = lane == 0 ? su : lane == 1 ? sv : lane == 2 ? sa : lane == 3 ? sbt : lane == 4 ? sc
                                : lane == 5 ? so : lane == 6 ? sr : lane == 7 ? sg : lane == 8 ? sbl : sm;
                        if (lane < DREC) atomicAdd(d_rec + (size_t)r * DREC + lane, v);
                        else if (lane == DREC) atomicAdd(d_masks + g, v);
                    } else if (lane == 0) {
                        atomicAdd(d_masks + g, sm);
                    }
                }
            }
        }
        if (!queue) break;
    }
}

template <int TW, int TH, int PPT>
void launch_fwd_t(hipStream_t s, int num_cus, const float* rec, const uint32_t* vals, const uint32_t* ranges,
                  const ViewSet& views, const DevSettings& st, float* images, float* t_final, int32_t* last,
                  int32_t* examined, int32_t* stats, uint32_t* queue) {
    int grid = (int)views.total_tiles;
    if (queue) {
        static int full = 0;
        if (!full) full = persistent_grid(composite_fwd_kernel<TW, TH, PPT>, TW * TH / PPT, num_cus);
        grid = min(full, grid);
    }
    hipLaunchKernelGGL((composite_fwd_kernel<TW, TH, PPT>), dim3(grid), dim3(TW * TH / PPT), 0, s,
                       reinterpret_cast<const float4*>(rec), vals, reinterpret_cast<const uint2*>(ranges), views, st,
                       images, t_final, last, examined, reinterpret_cast<int4*>(stats), queue);
}

template <int TW, int TH, int PPT>
void launch_bwd_t(hipStream_t s, int num_cus, const float* rec, const uint32_t* vals, const uint32_t* ranges,
                  const ViewSet& views, const DevSettings& st, const float* t_final, const int32_t* last,
                  const float* dl, int64_t n, float* d_rec, float* d_masks, uint32_t* queue) {
    int grid = (int)views.total_tiles;
    if (queue) {
        static int full = 0;
        if (!full) full = persistent_grid(composite_bwd_kernel<TW, TH, PPT>, TW * TH / PPT, num_cus);
        grid = min(full, grid);
    }
    hipLaunchKernelGGL((composite_bwd_kernel<TW, TH, PPT>), dim3(grid), dim3(TW * TH / PPT), 0, s,
                       reinterpret_cast<const float4*>(rec), vals, reinterpret_cast<const uint2*>(ranges), views, st,
                       t_final, last, dl, n, d_rec, d_masks, queue);
}

// The supported (tile_w, tile_h, pixels per thread) shapes.
#define MGS_COMPOSITE_SHAPES(X) \
    X(8, 8, 1)                  \
    X(16, 8, 1)                 \
    X(16, 8, 2)                 \
    X(16, 16, 1)                \
    X(16, 16, 2)                \
    X(16, 16, 4)                \
    X(32, 8, 1)                 \
    X(32, 8, 2)                 \
    X(32, 8, 4)

}  // namespace

bool composite_config_supported(const CompositeConfig& c) {
#define MGS_MATCH(A, B, P) \
    if (c.tile_w == A && c.tile_h == B && c.ppt == P) return true;
    MGS_COMPOSITE_SHAPES(MGS_MATCH)
#undef MGS_MATCH
    return false;
}

void launch_composite_fwd(hipStream_t stream, const CompositeConfig& cfg, const float* rec, const uint32_t* vals,
                          const uint32_t* ranges, const ViewSet& views, const DevSettings& st, float* images,
                          float* t_final, int32_t* last, int32_t* examined, int32_t* stats, uint32_t* queue,
                          int num_cus) {
    if (views.total_tiles == 0) return;
#define MGS_FWD(A, B, P)                                                                                     \
    if (cfg.tile_w == A && cfg.tile_h == B && cfg.ppt == P) {                                                \
        launch_fwd_t<A, B, P>(stream, num_cus, rec, vals, ranges, views, st, images, t_final, last, examined, stats, \
                              queue);                                                                        \
        return;                                                                                              \
    }
    MGS_COMPOSITE_SHAPES(MGS_FWD)
#undef MGS_FWD
}

void launch_composite_bwd(hipStream_t stream, const CompositeConfig& cfg, const float* rec, const uint32_t* vals,
                          const uint32_t* ranges, const ViewSet& views, const DevSettings& st, const float* t_final,
                          const int32_t* last, const float* dl_dimages, int64_t n, float* d_rec, float* d_masks,
                          uint32_t* queue, int num_cus) {
    if (views.total_tiles == 0) return;
#define MGS_BWD(A, B, P)                                                                                        \
    if (cfg.tile_w == A && cfg.tile_h == B && cfg.ppt == P) {                                                   \
        launch_bwd_t<A, B, P>(stream, num_cus, rec, vals, ranges, views, st, t_final, last, dl_dimages, n, d_rec, \
                              d_masks, queue);                                                                  \
        return;                                                                                                 \
    }
    MGS_COMPOSITE_SHAPES(MGS_BWD)
#undef MGS_BWD
}

}  // namespace mgs
