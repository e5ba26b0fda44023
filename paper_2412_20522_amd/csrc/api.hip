// Host side of the C ABI declared in include/maskgs.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "maskgs.h"

using namespace mgs;

struct mgs_ctx {
    int device = 0;
    int num_cus = 256;
    void* scan_noalloc = nullptr;  // this device's address of the scratch of mgs_scan_noalloc
    std::string err;
    // per-stage timing
    bool prof_on = false;
    struct Rec {
        int stage;
        hipEvent_t a, b;
    };
    std::vector<Rec> prof;
    std::vector<hipEvent_t> pool;
    ~mgs_ctx() {
        for (auto& r : prof) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        for (auto e : pool) (void)hipEventDestroy(e);
    }
    hipEvent_t take_event() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
};

namespace {

// Brackets the launches of one stage with two events while profiling is on.
struct StageTimer {
    mgs_ctx* ctx;
    hipStream_t stream;
    int stage;
    hipEvent_t a = nullptr;
    StageTimer(mgs_ctx* c, hipStream_t s, int st) : ctx(c), stream(s), stage(st) {
        if (ctx && ctx->prof_on) {
            a = ctx->take_event();
            if (a) (void)hipEventRecord(a, stream);
        }
    }
    ~StageTimer() {
        if (!a) return;
        hipEvent_t b = ctx->take_event();
        if (!b) {
            ctx->pool.push_back(a);
            return;
        }
        (void)hipEventRecord(b, stream);
        ctx->prof.push_back({stage, a, b});
    }
};

thread_local std::string g_create_error;

mgs_status fail(mgs_ctx* ctx, mgs_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    else g_create_error = buf;
    return s;
}

#define MGS_HIP(ctx, call)                                                                          \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess) return fail((ctx), MGS_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

#define MGS_CHECK_LAUNCH(ctx)                                                                          \
    do {                                                                                              \
        hipError_t e_ = hipGetLastError();                                                            \
        if (e_ != hipSuccess) return fail((ctx), MGS_ERR_HIP, "kernel launch: %s", hipGetErrorString(e_)); \
    } while (0)

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};

// Grows a device buffer (contents are not preserved).
mgs_status grow(mgs_ctx* ctx, DevBuf& b, size_t need) {
    if (need <= b.bytes && b.p) return MGS_OK;
    if (b.p) {
        (void)hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
    }
    size_t want = need + need / 4 + 256;
    want = (want + 255) & ~(size_t)255;
    if (hipMalloc(&b.p, want) != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return fail(ctx, MGS_ERR_OOM, "hipMalloc of %zu bytes failed", want);
    }
    b.bytes = want;
    return MGS_OK;
}

void release(DevBuf& b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

bool valid_tile(int w, int h) {
    return (w == 8 && h == 8) || (w == 16 && h == 8) || (w == 16 && h == 16) || (w == 32 && h == 8);
}

mgs_status check_settings(mgs_ctx* ctx, const mgs_settings* st) {
    if (!st) return fail(ctx, MGS_ERR_INVALID_ARG, "settings is NULL");
    if (!valid_tile(st->tile_w, st->tile_h))
        return fail(ctx, MGS_ERR_INVALID_ARG, "tile %dx%d not one of 8x8, 16x8, 16x16, 32x8", st->tile_w, st->tile_h);
    const int bd = st->batch_depth;
    if (!(bd == 32 || bd == 64 || bd == 128 || bd == 256) || bd > st->tile_w * st->tile_h * 4)
        return fail(ctx, MGS_ERR_INVALID_ARG, "batch_depth %d not one of 32, 64, 128, 256", bd);
    if (st->sh_degree < 0 || st->sh_degree > 3) return fail(ctx, MGS_ERR_INVALID_ARG, "sh_degree %d", st->sh_degree);
    const CompositeConfig cf{st->tile_w, st->tile_h, st->fwd_ppt}, cb{st->tile_w, st->tile_h, st->bwd_ppt};
    if (!composite_config_supported(cf) || !composite_config_supported(cb))
        return fail(ctx, MGS_ERR_UNSUPPORTED, "pixels per thread %d/%d unsupported for tile %dx%d", st->fwd_ppt,
                    st->bwd_ppt, st->tile_w, st->tile_h);
    if (!(st->alpha_max > 0.f && st->alpha_max < 1.f)) return fail(ctx, MGS_ERR_INVALID_ARG, "alpha_max in (0, 1)");
    if (!(st->near_plane > 0.f)) return fail(ctx, MGS_ERR_INVALID_ARG, "near_plane must be > 0");
    if (st->mask_mode != MGS_MASK_RASTER && st->mask_mode != MGS_MASK_OPACITY)
        return fail(ctx, MGS_ERR_INVALID_ARG, "mask_mode %d not MGS_MASK_RASTER or MGS_MASK_OPACITY", st->mask_mode);
    return MGS_OK;
}

mgs_status check_cameras(mgs_ctx* ctx, const mgs_camera* cams, int n_views) {
    if (n_views < 1 || n_views > MGS_MAX_VIEWS)
        return fail(ctx, MGS_ERR_INVALID_ARG, "n_views %d not in [1, %d]", n_views, MGS_MAX_VIEWS);
    if (!cams) return fail(ctx, MGS_ERR_INVALID_ARG, "cams is NULL");
    int64_t pixels = 0;
    for (int v = 0; v < n_views; ++v) {
        const mgs_camera& c = cams[v];
        if (c.width <= 0 || c.height <= 0 || c.width > 16384 || c.height > 16384)
            return fail(ctx, MGS_ERR_INVALID_ARG, "view %d: size %dx%d", v, c.width, c.height);
        if (!(c.fx > 0.f && c.fy > 0.f)) return fail(ctx, MGS_ERR_INVALID_ARG, "view %d: focal lengths", v);
        pixels += (int64_t)c.width * c.height;
    }
    // per-view pixel offsets are 32-bit
    if (pixels > (int64_t)0xffffffffll)
        return fail(ctx, MGS_ERR_INVALID_ARG, "%lld pixels over all views exceed 2^32 - 1", (long long)pixels);
    return MGS_OK;
}

mgs_status check_gaussians(mgs_ctx* ctx, const mgs_gaussians* g, bool need_masks) {
    if (!g) return fail(ctx, MGS_ERR_INVALID_ARG, "gaussians is NULL");
    if (g->n < 0 || g->n > (int64_t)0x7fffffff) return fail(ctx, MGS_ERR_INVALID_ARG, "n = %lld", (long long)g->n);
    if (g->n > 0 && (!g->means || !g->log_scales || !g->quats || !g->opacity_logits || !g->sh ||
                     (need_masks && !g->masks)))
        return fail(ctx, MGS_ERR_INVALID_ARG, "a Gaussian parameter pointer is NULL");
    if (g->n > 0 && (((uintptr_t)g->quats & 15) != 0))
        return fail(ctx, MGS_ERR_INVALID_ARG, "quats must be 16-byte aligned");
    return MGS_OK;
}

// Host-side construction of the per-view device constants.
ViewSet make_views(const mgs_camera* cams, int n_views, int tw, int th, int64_t* total_px, int wide_tiles = -1) {
    ViewSet vs;
    memset(&vs, 0, sizeof vs);
    vs.n_views = n_views;
    uint32_t toff = 0, poff = 0, roff = 0;
    for (int i = 0; i < n_views; ++i) {
        const mgs_camera& c = cams[i];
        DevView& d = vs.v[i];
        for (int r = 0; r < 3; ++r) {
            for (int k = 0; k < 3; ++k) d.W[3 * r + k] = c.viewmat[4 * r + k];
            d.t[r] = c.viewmat[4 * r + 3];
        }
        d.fx = c.fx; d.fy = c.fy; d.cx = c.cx; d.cy = c.cy;
        for (int k = 0; k < 3; ++k) {
            double s = 0.0;
            for (int r = 0; r < 3; ++r) s += (double)c.viewmat[4 * r + k] * (double)c.viewmat[4 * r + 3];
            d.campos[k] = (float)(-s);
        }
        d.width = c.width;
        d.height = c.height;
        d.grid_w = (c.width + tw - 1) / tw;
        d.grid_h = (c.height + th - 1) / th;
        d.tile_off = toff;
        d.px_off = poff;
        // records covering more tiles than wide_min are listed per region
        if (wide_tiles < 0) d.wide_min = 0xffffffffu;
        else if (wide_tiles > 0) d.wide_min = (uint32_t)wide_tiles;
        else d.wide_min = 64u;
        d.reg_w = (d.grid_w + REGION - 1) / REGION;
        d.reg_h = (d.grid_h + REGION - 1) / REGION;
        d.reg_off = roff;
        toff += (uint32_t)(d.grid_w * d.grid_h);
        poff += (uint32_t)(c.width * c.height);
        roff += (uint32_t)(d.reg_w * d.reg_h);
    }
    vs.total_tiles = toff;
    vs.total_regions = roff;
    if (total_px) *total_px = poff;
    return vs;
}

void set_limits(ViewSet& vs, const mgs_camera* cams, float jac_clamp) {
    for (int i = 0; i < vs.n_views; ++i) {
        vs.v[i].limx = (float)((double)jac_clamp * 0.5 * cams[i].width / cams[i].fx);
        vs.v[i].limy = (float)((double)jac_clamp * 0.5 * cams[i].height / cams[i].fy);
    }
}

DevSettings make_settings(const mgs_settings* s) {
    DevSettings d;
    d.tile_w = s->tile_w;
    d.tile_h = s->tile_h;
    d.batch = s->batch_depth;
    d.sh_degree = s->sh_degree;
    d.alpha_max = s->alpha_max;
    d.near_plane = s->near_plane;
    d.dilation = s->dilation;
    d.lambda_floor = s->lambda_floor;
    d.bg[0] = s->bg[0]; d.bg[1] = s->bg[1]; d.bg[2] = s->bg[2];
    if (s->exact_mode) {
        d.alpha_min = 0.f;
        d.t_min = 0.f;
        d.q_max = INFINITY;
        d.full_rect = 1;
        d.tile_cull = 0;
    } else {
        d.alpha_min = s->alpha_min;
        d.t_min = s->t_min;
        d.q_max = s->q_max;
        d.full_rect = 0;
        d.tile_cull = s->tile_cull != 0;
    }
    d.qs_max = (float)(-0.5 / std::log(2.0) * (double)d.q_max);
    d.mask_opacity = s->mask_mode == MGS_MASK_OPACITY;
    return d;
}

int bits_for(uint64_t v) {  // bits needed to hold values < v
    int b = 0;
    while (b < 64 && (1ull << b) < v) ++b;
    return b;
}

}  // namespace

struct mgs_frame {
    mgs_ctx* ctx = nullptr;
    // state of the last forward
    bool have_forward = false;
    mgs_gaussians g{};
    ViewSet views{};
    DevSettings st{};
    CompositeConfig cfg_fwd{}, cfg_bwd{};
    int persistent = 0;
    int n_views = 0;
    int64_t n = 0, R = 0, P = 0, K = 0, W = 0, total_tiles = 0, capacity = 0;
    int sort_passes = 0, tile_bits = 0;
    bool sorted_in_alt = false, order_in_alt = false;
    // fixed workspace (mgs_frame_reserve): no allocation, no synchronisation
    bool reserved = false;
    int64_t res_R = 0, res_P = 0, res_T = 0, K_cap = 0, cur_cap = 0, stg_cap = 0;
    // device buffers: per record, then per list entry (32-bit cell keys), per
    // tile and region, per pixel
    DevBuf rec, srec, depth, tiles, rkeys, rvals, rkeys_alt, rvals_alt, cnt_sorted, tmask,
        cls_part;
    // order, order_b: the tile orders of the forward and the backward
    // compositing (most expensive first), tcost: the forward's cost keys,
    // caps: checkpoint totals per workgroup of 256 tiles
    DevBuf keys, vals, keys_alt, vals_alt, ranges, caps, tcost, order, order_b, cur_off, nbatch, cur, cur_stg, stg,
        t_final, last, stats, evals;
    bool have_stats = false;  // the last forward wrote the per-pixel work counters
    DevBuf d_rec, dm_acc, rsort_tmp, sort_tmp, misc, queue, sum_tmp;  // d_rec, dm_acc: FP64
    DevBuf imp_acc;  // FP64 sums of the importance forward
    // d_rec is all zeros from the forward compositing (which clears it) to
    // the backward that accumulates into it; false after a backward and
    // after (re)allocation (a backward then fills it first)
    bool drec_zero = false;
    // views of the last forward, whose per-tile batch counts (nbatch) order
    // the tiles of the next forward over the same views
    ViewSet order_views{};
    bool order_valid = false;
    // the last forward ordered its tiles by measured batch counts (those of
    // the forward before it over the same views); the backward then reuses
    // that order
    bool fwd_order_measured = false;
    // misc: flags (u32) at 0, list entry count (u64) at 8, wide record count
    // (u64) at 16, checkpoint count (u64) at 24, region entry count (u64) at
    // 32, staged-entry counter (u32) at 192; the tile orders' histogram and
    // cursors (2 x 256 u32) from 256
    uint64_t* h_pinned = nullptr;  // read-back of misc
    uint32_t* keys_sorted() { return (uint32_t*)(sorted_in_alt ? keys_alt.p : keys.p); }
    uint32_t* vals_sorted() { return (uint32_t*)(sorted_in_alt ? vals_alt.p : vals.p); }
    uint32_t* record_order() { return (uint32_t*)(order_in_alt ? rvals_alt.p : rvals.p); }
    uint32_t* flags() { return (uint32_t*)misc.p; }
    uint64_t* total() { return (uint64_t*)((char*)misc.p + 8); }
    uint64_t* wide_counts() { return (uint64_t*)((char*)misc.p + 16); }
    uint64_t* cur_need() { return (uint64_t*)((char*)misc.p + 24); }
    uint32_t* stg_count() { return (uint32_t*)((char*)misc.p + 192); }
    uint32_t* order_hist() { return (uint32_t*)((char*)misc.p + 256); }
    HybridBuffers hybrid(bool clear_drec = false) {
        const uint64_t cap = reserved ? (uint64_t)cur_cap : (uint64_t)std::min(cur.bytes / 16, cur_stg.bytes / 8);
        const uint64_t scap = reserved ? (uint64_t)stg_cap : (uint64_t)(stg.bytes / 8);
        // pairs of doubles covering the R x DREC accumulator (the allocation
        // has 8 bytes of slack for an odd count)
        const uint64_t n2 = clear_drec ? ((uint64_t)R * DREC + 1) / 2 : 0;
        return HybridBuffers{vals_sorted(), (const uint32_t*)ranges.p, (uint32_t*)cur.p, (const uint32_t*)cur_off.p, (uint32_t*)nbatch.p, cur_need(), cap,
                             flags(), (uint32_t*)cur_stg.p, (uint32_t*)stg.p, stg_count(), scap,
                             clear_drec ? (double*)d_rec.p : nullptr, n2, (const uint32_t*)order.p};
    }
};

extern "C" {

int mgs_version(void) { return 200; }

mgs_status mgs_default_settings(mgs_settings* out) {
    if (!out) return MGS_ERR_INVALID_ARG;
    memset(out, 0, sizeof *out);
    out->tile_w = 16;
    out->tile_h = 16;
    out->batch_depth = 256;
    out->sh_degree = 3;
    out->alpha_min = 1.f / 255.f;
    out->alpha_max = 0.99f;
    out->t_min = 1e-4f;
    out->q_max = 9.f;
    out->near_plane = 0.2f;
    out->dilation = 0.3f;
    out->jac_clamp = 1.3f;
    out->lambda_floor = 0.1f;
    out->exact_mode = 0;
    out->persistent = 0;
    out->fwd_ppt = 2;
    out->bwd_ppt = 2;
    out->wide_tiles = 0;
    out->stats = 1;
    out->tile_cull = 1;
    return MGS_OK;
}

mgs_status mgs_create(int device, mgs_ctx** out) {
    if (!out) return fail(nullptr, MGS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0)
        return fail(nullptr, MGS_ERR_HIP, "no HIP device available");
    if (device < 0 || device >= count) return fail(nullptr, MGS_ERR_INVALID_ARG, "device %d of %d", device, count);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return fail(nullptr, MGS_ERR_HIP, "device properties");
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(nullptr, MGS_ERR_UNSUPPORTED, "device %d is %s; this library is built for gfx950", device,
                    prop.gcnArchName);
    if (hipSetDevice(device) != hipSuccess) return fail(nullptr, MGS_ERR_HIP, "hipSetDevice(%d)", device);
    void* noalloc = nullptr;
    const hipError_t ne = scan_noalloc_init(device, &noalloc);
    if (ne != hipSuccess)
        return fail(nullptr, MGS_ERR_HIP, "address of the scan scratch: %s", hipGetErrorString(ne));
    mgs_ctx* c = new (std::nothrow) mgs_ctx();
    if (!c) return fail(nullptr, MGS_ERR_OOM, "context allocation");
    c->device = device;
    c->scan_noalloc = noalloc;
    c->num_cus = prop.multiProcessorCount;
    *out = c;
    return MGS_OK;
}

mgs_status mgs_destroy(mgs_ctx* ctx) {
    delete ctx;
    return MGS_OK;
}

const char* mgs_last_error(const mgs_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

mgs_status mgs_frame_create(mgs_ctx* ctx, mgs_frame** out) {
    if (!ctx || !out) return fail(ctx, MGS_ERR_INVALID_ARG, "NULL argument");
    mgs_frame* f = new (std::nothrow) mgs_frame();
    if (!f) return fail(ctx, MGS_ERR_OOM, "frame allocation");
    f->ctx = ctx;
    if (hipHostMalloc((void**)&f->h_pinned, 256, hipHostMallocDefault) != hipSuccess) {
        delete f;
        return fail(ctx, MGS_ERR_OOM, "pinned host allocation");
    }
    if (grow(ctx, f->misc, 256 + 2048) != MGS_OK) {
        (void)hipHostFree(f->h_pinned);
        delete f;
        return MGS_ERR_OOM;
    }
    *out = f;
    return MGS_OK;
}

mgs_status mgs_frame_destroy(mgs_frame* f) {
    if (!f) return MGS_OK;
    (void)hipDeviceSynchronize();
    DevBuf* bufs[] = {&f->rec,      &f->srec,      &f->depth,     &f->tiles,     &f->rkeys,    &f->rvals,
                      &f->rkeys_alt, &f->rvals_alt, &f->cnt_sorted, &f->tmask, &f->cls_part,
                      &f->keys,     &f->vals,      &f->keys_alt, &f->vals_alt,  &f->ranges,
                      &f->caps,     &f->tcost,     &f->order,     &f->order_b,   &f->cur_off,   &f->nbatch,   &f->cur,       &f->cur_stg,   &f->stg,
                      &f->t_final,  &f->last,
                      &f->stats,    &f->evals,     &f->d_rec,     &f->dm_acc,    &f->rsort_tmp, &f->sort_tmp,
                      &f->misc,     &f->queue,     &f->sum_tmp,  &f->imp_acc};
    for (DevBuf* b : bufs) release(*b);
    if (f->h_pinned) (void)hipHostFree(f->h_pinned);
    delete f;
    return MGS_OK;
}

mgs_status mgs_frame_get_stats(const mgs_frame* f, mgs_frame_stats* out) {
    if (!f || !out) return MGS_ERR_INVALID_ARG;
    out->n_gaussians = f->n;
    out->n_views = f->n_views;
    out->n_records = f->R;
    out->n_pixels = f->P;
    out->n_instances = f->K;
    out->total_tiles = f->total_tiles;
    out->instance_capacity = f->capacity;
    out->n_wide = f->W;
    out->sort_passes = f->sort_passes;
    out->tile_bits = f->tile_bits;
    return MGS_OK;
}

// Grows the per-tile batch counts; a new allocation holds no counts of an
// earlier forward.
static mgs_status grow_nbatch(mgs_frame* f, size_t bytes) {
    const size_t before = f->nbatch.p ? f->nbatch.bytes : 0;
    const mgs_status s = grow(f->ctx, f->nbatch, bytes);
    if (s != MGS_OK || f->nbatch.bytes != before) f->order_valid = false;
    return s;
}

// Grows the FP64 per-record gradient accumulator; a new allocation is not
// known to be zero.
static mgs_status grow_drec(mgs_frame* f) {
    const size_t before = f->d_rec.p ? f->d_rec.bytes : 0;  // grow reallocates only to a larger size
    const mgs_status s = grow(f->ctx, f->d_rec, (size_t)f->R * DREC * 8 + 8);
    if (s != MGS_OK || f->d_rec.bytes != before) f->drec_zero = false;
    return s;
}

mgs_status mgs_frame_reserve(mgs_frame* f, mgs_stream stream_, double slack) {
    if (!f) return MGS_ERR_INVALID_ARG;
    mgs_ctx* ctx = f->ctx;
    hipStream_t stream = (hipStream_t)stream_;
    if (slack <= 0.0) {
        f->reserved = false;
        return MGS_OK;
    }
    if (!(slack >= 1.0)) return fail(ctx, MGS_ERR_INVALID_ARG, "slack %g must be >= 1 (or <= 0 to release)", slack);
    if (!f->have_forward || f->reserved)
        return fail(ctx, MGS_ERR_STATE, "mgs_frame_reserve needs a preceding plain mgs_forward");
    MGS_HIP(ctx, hipMemcpyAsync(f->h_pinned, f->misc.p, 200, hipMemcpyDeviceToHost, stream));
    MGS_HIP(ctx, hipStreamSynchronize(stream));
    const double K = (double)f->h_pinned[1], C = (double)f->h_pinned[3];
    const double S = (double)(f->h_pinned[24] & 0xffffffffu);
    const int64_t K_cap = (int64_t)std::ceil(K * slack) + 4096;
    const int64_t cur_cap = (int64_t)std::ceil(C * slack) + 4096;
    const int64_t stg_cap = std::min<int64_t>((int64_t)std::ceil(S * slack) + 4096, 0xffffffffll);
    if (K_cap > (int64_t)0x7fffffff) return fail(ctx, MGS_ERR_CAPACITY, "instance capacity beyond 2^31 - 1");
    mgs_status s;
    const size_t kb = (size_t)K_cap * 4 + 16;
    if ((s = grow(ctx, f->keys, kb)) || (s = grow(ctx, f->vals, kb)) || (s = grow(ctx, f->keys_alt, kb)) ||
        (s = grow(ctx, f->vals_alt, kb)) || (s = grow(ctx, f->sort_tmp, sort_scratch_bytes(K_cap))) ||
        (s = grow(ctx, f->cur, (size_t)cur_cap * 16 + 16)) || (s = grow_drec(f)) || (s = grow(ctx, f->dm_acc, (size_t)f->n * 8 + 8)) ||
        (s = grow(ctx, f->cur_stg, (size_t)cur_cap * 8 + 8)) || (s = grow(ctx, f->stg, (size_t)stg_cap * 8 + 8)))
        return s;
    f->stg_cap = stg_cap;
    f->K_cap = K_cap;
    f->cur_cap = cur_cap;
    f->res_R = f->R;
    f->res_P = f->P;
    f->res_T = f->total_tiles;
    f->reserved = true;
    return MGS_OK;
}

mgs_status mgs_frame_check(mgs_frame* f, mgs_stream stream_) {
    if (!f) return MGS_ERR_INVALID_ARG;
    mgs_ctx* ctx = f->ctx;
    hipStream_t stream = (hipStream_t)stream_;
    if (!f->have_forward) return fail(ctx, MGS_ERR_STATE, "no forward on this frame");
    MGS_HIP(ctx, hipMemcpyAsync(f->h_pinned, f->misc.p, 32, hipMemcpyDeviceToHost, stream));
    MGS_HIP(ctx, hipStreamSynchronize(stream));
    const uint32_t flags = (uint32_t)(f->h_pinned[0] & 0xffffffffu);
    const uint64_t K = f->h_pinned[1], W = f->h_pinned[2], C = f->h_pinned[3];
    f->W = (int64_t)W;
    if (f->reserved) f->K = (int64_t)std::min<uint64_t>(K, (uint64_t)f->K_cap);
    if (flags & FLAG_NONFINITE) return fail(ctx, MGS_ERR_NONFINITE, "non-finite projected geometry");
    if (flags & FLAG_CAPACITY)
        return fail(ctx, MGS_ERR_CAPACITY,
                    "the last forward exceeded its workspace: %llu list entries (capacity %lld), %llu checkpoints "
                    "(%lld)",
                    (unsigned long long)K, (long long)f->K_cap, (unsigned long long)C, (long long)f->cur_cap);
    return MGS_OK;
}

namespace {
mgs_status forward_impl(mgs_frame* f, mgs_stream stream_, const mgs_gaussians* g, const mgs_camera* cams, int n_views,
                        const mgs_settings* st, float* images, float* t_final_out, float* imp_sum, float* imp_max) {
    if (!f) return MGS_ERR_INVALID_ARG;
    mgs_ctx* ctx = f->ctx;
    hipStream_t stream = (hipStream_t)stream_;
    mgs_status s;
    if ((s = check_gaussians(ctx, g, true)) != MGS_OK) return s;
    if ((s = check_cameras(ctx, cams, n_views)) != MGS_OK) return s;
    if ((s = check_settings(ctx, st)) != MGS_OK) return s;
    if (!images) return fail(ctx, MGS_ERR_INVALID_ARG, "images is NULL");
    // record ids (view * n + Gaussian) are 32-bit
    if (g->n * (int64_t)n_views > (int64_t)0xffffffffll)
        return fail(ctx, MGS_ERR_INVALID_ARG, "%lld records (views x Gaussians) exceed 2^32 - 1",
                    (long long)(g->n * (int64_t)n_views));
    f->have_forward = false;
    f->g = *g;
    f->n = g->n;
    f->n_views = n_views;
    f->R = g->n * n_views;
    f->views = make_views(cams, n_views, st->tile_w, st->tile_h, &f->P, st->wide_tiles);
    set_limits(f->views, cams, st->jac_clamp);
    f->st = make_settings(st);
    f->cfg_fwd = CompositeConfig{st->tile_w, st->tile_h, st->fwd_ppt};
    f->cfg_bwd = CompositeConfig{st->tile_w, st->tile_h, st->bwd_ppt};
    f->persistent = st->persistent;
    f->total_tiles = f->views.total_tiles;
    const int64_t R = f->R, P = f->P, T = f->total_tiles, NR = f->views.total_regions;
    f->tile_bits = bits_for((uint64_t)(T + NR));
    if (f->reserved && (R > f->res_R || P > f->res_P || T > f->res_T))
        return fail(ctx, MGS_ERR_CAPACITY,
                    "records %lld, pixels %lld or tiles %lld exceed the reserved workspace (%lld, %lld, %lld)",
                    (long long)R, (long long)P, (long long)T, (long long)f->res_R, (long long)f->res_P,
                    (long long)f->res_T);
    if ((s = grow(ctx, f->rec, (size_t)R * 48 + 16)) || (s = grow(ctx, f->srec, (size_t)R * 48 + 16)) ||
        (s = grow(ctx, f->depth, (size_t)R * 4 + 4)) ||
        (s = grow(ctx, f->tiles, (size_t)R * 4 + 4)) ||
        (s = grow(ctx, f->rkeys, (size_t)R * 8 + 16)) || (s = grow(ctx, f->rvals, (size_t)R * 4 + 16)) ||
        (s = grow(ctx, f->rkeys_alt, (size_t)R * 8 + 16)) || (s = grow(ctx, f->rvals_alt, (size_t)R * 4 + 16)) ||
        (s = grow(ctx, f->cnt_sorted, (size_t)R * 4 + 4)) ||
        (s = grow(ctx, f->tmask, (size_t)R * 8 + 8)) ||
        (s = grow(ctx, f->cls_part, classify_parts_bytes(R))) ||
        (s = grow(ctx, f->ranges, (size_t)(T + NR) * 8)) || (s = grow(ctx, f->caps, (size_t)T * 4 + 4)) ||
        (s = grow(ctx, f->tcost, (size_t)T * 4 + 4)) || (s = grow(ctx, f->order, (size_t)T * 4 + 4)) ||
        (s = grow(ctx, f->order_b, (size_t)T * 4 + 4)) ||
        (s = grow(ctx, f->cur_off, (size_t)T * 4 + 4)) || (s = grow_nbatch(f, (size_t)T * 4 + 4)) ||
        (s = grow(ctx, f->t_final, (size_t)P * 4)) || (s = grow(ctx, f->last, (size_t)P * 4)) ||
        (s = grow(ctx, f->stats, (size_t)P * 16)) || (s = grow(ctx, f->evals, (size_t)P * 16)) ||
        (s = grow(ctx, f->rsort_tmp, sort_scratch_bytes(R))) || (s = grow(ctx, f->queue, 256)))
        return s;
    launch_fill_u32(stream, f->flags(), 10, 0u);  // flags and the counters up to byte 40
    {
        StageTimer t(ctx, stream, MGS_STAGE_PROJECT);
        // the radius stays in the records (B.w); the export reads it there
        launch_project_fwd(stream, *g, f->views, f->st, (float*)f->rec.p, (float*)f->depth.p, nullptr,
                           (uint32_t*)f->tiles.p, f->flags(), (uint32_t*)f->rkeys.p, (uint32_t*)f->rvals.p);
    }
    {
        // records in (view, depth, record) order, those without tiles last in
        // their view; then the sorted record copy, list entry counts and wide
        // flags in that order
        StageTimer t(ctx, stream, MGS_STAGE_DEPTH_SORT);
        // 32-bit depth keys (written by the projection) sorted within each
        // view's segment of n records: the order of 64-bit (view, depth) keys
        // in 4 passes instead of 5
        bool alt = false;
        launch_radix_sort_segmented(stream, (uint32_t*)f->rkeys.p, (uint32_t*)f->rvals.p, (uint32_t*)f->rkeys_alt.p,
                                    (uint32_t*)f->rvals_alt.p, R, f->n, f->rsort_tmp.p, &alt);
        f->order_in_alt = alt;
        launch_permute_classify(stream, f->record_order(),
                                (const uint32_t*)(f->order_in_alt ? f->rkeys_alt.p : f->rkeys.p),
                                (const float*)f->rec.p, R, f->n, f->views, f->st,
                                (uint32_t*)f->cnt_sorted.p,
                                (uint64_t*)f->tmask.p, (float*)f->srec.p,
                                (uint32_t*)f->cls_part.p);
    }
    {
        // list offsets: one scan over the classification's per-workgroup
        // counts; the duplication adds the counts within its workgroup
        StageTimer t(ctx, stream, MGS_STAGE_SCAN);
        launch_list_offsets(stream, (uint32_t*)f->cls_part.p, R, f->total(), f->wide_counts());
    }
    MGS_CHECK_LAUNCH(ctx);
    const int64_t B = st->batch_depth;
    const uint64_t* K_dev = nullptr;  // live instance count on the device (fixed workspace)
    if (f->reserved) {
        // no synchronisation: the sort, ranges and compositing take the live
        // counts from the device and the capacities from the reservation;
        // overflows raise device flags, read by mgs_frame_check
        f->K = f->K_cap;
        K_dev = f->total();
    } else {
        // the one synchronisation of the plain path: the list entry counts
        // size the sort and the batch checkpoints
        MGS_HIP(ctx, hipMemcpyAsync(f->h_pinned, f->misc.p, 200, hipMemcpyDeviceToHost, stream));
        MGS_HIP(ctx, hipStreamSynchronize(stream));
        const uint32_t flags = (uint32_t)(f->h_pinned[0] & 0xffffffffu);
        const uint64_t K = f->h_pinned[1];
        const uint64_t W = f->h_pinned[2], KW = f->h_pinned[4];
        if (flags & FLAG_NONFINITE) return fail(ctx, MGS_ERR_NONFINITE, "non-finite projected geometry");
        if (K > (uint64_t)0x7fffffff) return fail(ctx, MGS_ERR_CAPACITY, "%llu list entries exceed 2^31 - 1",
                                                    (unsigned long long)K);
        f->K = (int64_t)K;
        f->W = (int64_t)W;
        // checkpoints: per tile 2 (ceil(narrow / B) + ceil(region / B)) + 2,
        // and a region list is read by at most REGION^2 tiles
        const int64_t cur_bound =
            2 * ((f->K + B - 1) / B + T) + 2 * (((int64_t)KW * REGION * REGION + B - 1) / B + T) + 2 * T;
        if ((s = grow(ctx, f->keys, (size_t)K * 4 + 16)) || (s = grow(ctx, f->vals, (size_t)K * 4 + 16)) ||
            (s = grow(ctx, f->keys_alt, (size_t)K * 4 + 16)) || (s = grow(ctx, f->vals_alt, (size_t)K * 4 + 16)) ||
            (s = grow(ctx, f->sort_tmp, sort_scratch_bytes(f->K))) ||
            (s = grow(ctx, f->cur, (size_t)cur_bound * 16 + 16)) ||
            (s = grow(ctx, f->cur_stg, (size_t)cur_bound * 8 + 8)))
            return s;
        // the entries staged for the backward: room for the previous forward's
        // count with a margin (a batch that does not fit is merged again)
        const uint64_t prev = f->h_pinned[24] & 0xffffffffu;
        const uint64_t want = std::min<uint64_t>(std::max<uint64_t>((uint64_t)P, prev + prev / 4), 0xffffffffull);
        // (the count includes the unused tails of the workgroups' chunks)
        if ((s = grow(ctx, f->stg, (size_t)want * 8 + 8))) return s;
    }
    f->capacity = (int64_t)std::min<size_t>(f->keys.bytes / 4, f->vals.bytes / 4);
    {
        StageTimer t(ctx, stream, MGS_STAGE_DUPLICATE);
        launch_duplicate_lists(stream, (const float*)f->srec.p, (const uint32_t*)f->cnt_sorted.p,
                               (const uint64_t*)f->tmask.p,
                               (uint32_t*)f->cls_part.p, R, f->n, f->views, f->st, (uint32_t*)f->keys.p,
                               (uint32_t*)f->vals.p, f->K, f->flags());
    }
    // entries are already in (depth, record) order: a stable sort on the cell
    // bits alone gives the (cell, depth, record) order
    f->sort_passes = f->K > 1 ? (f->tile_bits + 7) / 8 : 0;
    bool in_alt = false;
    {
        StageTimer t(ctx, stream, MGS_STAGE_SORT);
        launch_radix_sort32(stream, (uint32_t*)f->keys.p, (uint32_t*)f->vals.p, (uint32_t*)f->keys_alt.p,
                            (uint32_t*)f->vals_alt.p, f->K, K_dev, 0, 8 * f->sort_passes, f->sort_tmp.p, &in_alt);
    }
    f->sorted_in_alt = in_alt;
    uint32_t* queue = f->persistent ? (uint32_t*)f->queue.p : nullptr;
    {
        StageTimer t(ctx, stream, MGS_STAGE_RANGES);
        // one launch clears the ranges, the tile order's histogram and
        // cursors, the staged-entry counter and the persistent queue
        const FillSpan zero[4] = {{(uint32_t*)f->ranges.p, 2 * (T + NR), 0u},
                                  {f->order_hist(), 512, 0u},
                                  {f->stg_count(), 1, 0u},
                                  {queue, 1, 0u}};
        launch_fill_spans(stream, zero, 4);
        launch_tile_ranges32(stream, f->keys_sorted(), f->K, K_dev, T + NR, (uint32_t*)f->ranges.p, true);
        // the forward takes the most expensive tiles first: by the batches the
        // last forward over the same views took, else by list length
        const bool measured = f->order_valid && std::memcmp(&f->order_views, &f->views, sizeof(ViewSet)) == 0;
        f->fwd_order_measured = measured;
        launch_tile_setup(stream, (const uint32_t*)f->ranges.p, f->views, (int)B,
                          measured ? (const uint32_t*)f->nbatch.p : nullptr, (uint32_t*)f->tcost.p,
                          (uint32_t*)f->cur_off.p, f->cur_need(), (uint32_t*)f->caps.p, f->order_hist(),
                          (uint32_t*)f->order.p);
    }
    const bool imp = imp_sum != nullptr;
    if (imp) {
        if ((s = grow(ctx, f->imp_acc, (size_t)f->n * 8 + 8))) return s;
        launch_fill_u32(stream, (uint32_t*)f->imp_acc.p, 2 * f->n, 0u);
        launch_fill_u32(stream, (uint32_t*)imp_max, f->n, 0u);
    }
    // the compositing clears the backward's accumulator (sized here; a fixed
    // workspace already holds it)
    if ((s = grow_drec(f))) return s;
    {
        StageTimer t(ctx, stream, MGS_STAGE_COMPOSITE_FWD);
        f->have_stats = st->stats != 0 && !imp;
        launch_hybrid_fwd(stream, f->cfg_fwd, (const float*)f->srec.p, f->hybrid(true), f->views, f->st, images,
                          (float*)f->t_final.p, (int32_t*)f->last.p, f->have_stats ? (int32_t*)f->stats.p : nullptr,
                          f->have_stats ? (int32_t*)f->evals.p : nullptr, queue, ctx->num_cus, f->n,
                          imp ? (double*)f->imp_acc.p : nullptr, imp ? (uint32_t*)imp_max : nullptr);
    }
    if (imp) launch_round_f64(stream, (const double*)f->imp_acc.p, imp_sum, f->n);
    MGS_CHECK_LAUNCH(ctx);
    if (t_final_out)
        MGS_HIP(ctx, hipMemcpyAsync(t_final_out, f->t_final.p, (size_t)P * 4, hipMemcpyDeviceToDevice, stream));
    f->drec_zero = true;
    f->have_forward = true;
    f->order_views = f->views;  // nbatch now holds this forward's batch counts
    f->order_valid = true;
    return MGS_OK;
}
}  // namespace

mgs_status mgs_forward(mgs_frame* f, mgs_stream stream, const mgs_gaussians* g, const mgs_camera* cams, int n_views,
                       const mgs_settings* st, float* images, float* t_final) {
    return forward_impl(f, stream, g, cams, n_views, st, images, t_final, nullptr, nullptr);
}

mgs_status mgs_forward_importance(mgs_frame* f, mgs_stream stream, const mgs_gaussians* g, const mgs_camera* cams,
                                  int n_views, const mgs_settings* st, float* images, float* t_final,
                                  float* imp_sum, float* imp_max) {
    if (!f) return MGS_ERR_INVALID_ARG;
    if (g && g->n > 0 && (!imp_sum || !imp_max))
        return fail(f->ctx, MGS_ERR_INVALID_ARG, "imp_sum and imp_max are required");
    if (g && g->n == 0) return forward_impl(f, stream, g, cams, n_views, st, images, t_final, nullptr, nullptr);
    return forward_impl(f, stream, g, cams, n_views, st, images, t_final, imp_sum, imp_max);
}

mgs_status mgs_backward(mgs_frame* f, mgs_stream stream_, const float* dl_dimages, const mgs_gradients* grads) {
    if (!f) return MGS_ERR_INVALID_ARG;
    mgs_ctx* ctx = f->ctx;
    hipStream_t stream = (hipStream_t)stream_;
    if (!f->have_forward) return fail(ctx, MGS_ERR_STATE, "mgs_backward without a preceding mgs_forward");
    if (!dl_dimages || !grads) return fail(ctx, MGS_ERR_INVALID_ARG, "NULL argument");
    if (grads->d_quats && ((uintptr_t)grads->d_quats & 15) != 0)
        return fail(ctx, MGS_ERR_INVALID_ARG, "d_quats must be 16-byte aligned");
    if (grads->accumulate != 0 && grads->accumulate != 1)
        return fail(ctx, MGS_ERR_INVALID_ARG, "accumulate must be 0 or 1");
    mgs_status s;
    // per-record 2D gradients and mask gradients accumulate in FP64: a wide
    // splat takes atomics from thousands of tiles whose partial sums cancel
    if ((s = grow_drec(f)) || (s = grow(ctx, f->dm_acc, (size_t)f->n * 8 + 8))) return s;
    uint32_t* queue = nullptr;
    if (!f->drec_zero) {
        // +0.0 in every double: normally the forward compositing has cleared
        // the accumulator; a second backward after one forward, or a new
        // allocation, fills it here
        launch_fill_u32(stream, (uint32_t*)f->d_rec.p, f->d_rec.bytes / 4, 0u);
    }
    f->drec_zero = false;  // this backward accumulates into it
    if (f->persistent) queue = (uint32_t*)f->queue.p;
    // the tile order: the forward's when it came from measured batch counts
    // (a scheduling choice: the order decides no result), else by this
    // forward's batch counts
    const bool own_order = !f->fwd_order_measured;
    {
        // one launch clears the FP64 mask gradients, the persistent queue and
        // the tile order's histogram and cursors
        const FillSpan zero[3] = {{(uint32_t*)f->dm_acc.p, 2 * f->n, 0u}, {queue, 1, 0u},
                                  {own_order ? f->order_hist() : nullptr, 512, 0u}};
        launch_fill_spans(stream, zero, 3);
    }
    HybridBuffers hb = f->hybrid();
    {
        StageTimer t(ctx, stream, MGS_STAGE_COMPOSITE_BWD);
        // the backward takes first the tiles where the forward took most
        // batches (the backward replays them)
        const uint32_t T = f->views.total_tiles;
        if (own_order) {
            launch_tile_order(stream, (const uint32_t*)f->nbatch.p, T, f->order_hist(), (uint32_t*)f->order_b.p,
                              true);
            hb.order = (const uint32_t*)f->order_b.p;
        } else {
            hb.order = (const uint32_t*)f->order.p;
        }
        launch_hybrid_bwd(stream, f->cfg_bwd, (const float*)f->srec.p, hb, f->views, f->st,
                          (const float*)f->t_final.p, (const int32_t*)f->last.p, dl_dimages, f->n,
                          (double*)f->d_rec.p, (double*)f->dm_acc.p, queue, ctx->num_cus);
    }
    {
        StageTimer t(ctx, stream, MGS_STAGE_PROJECT_BWD);
        launch_project_bwd64(stream, f->g, f->views, f->st, (double*)f->d_rec.p, (const double*)f->dm_acc.p,
                             *grads, (const uint32_t*)f->tiles.p);
    }
    MGS_CHECK_LAUNCH(ctx);
    return MGS_OK;
}

mgs_status mgs_autotune(mgs_frame* f, mgs_stream stream_, const mgs_gaussians* g, const mgs_camera* cams,
                        int n_views, const mgs_settings* base, float* images, const float* dl_dimages,
                        const mgs_gradients* grads, mgs_settings* best, double* best_ms) {
    if (!f || !best) return MGS_ERR_INVALID_ARG;
    mgs_ctx* ctx = f->ctx;
    hipStream_t stream = (hipStream_t)stream_;
    if (f->reserved) return fail(ctx, MGS_ERR_STATE, "mgs_autotune needs a frame without a fixed workspace");
    mgs_status s;
    if ((s = check_settings(ctx, base)) != MGS_OK) return s;
    if (!dl_dimages || !grads || !images) return fail(ctx, MGS_ERR_INVALID_ARG, "NULL argument");
    mgs_gradients gw = *grads;
    gw.accumulate = 0;  // every trial overwrites the gradients
    grads = &gw;
    const bool was_on = ctx->prof_on;
    ctx->prof_on = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        ctx->prof_on = was_on;
        return fail(ctx, MGS_ERR_HIP, "event creation");
    }
    // one warm-up and four timed forward + backward passes; the fastest counts
    auto trial = [&](const mgs_settings& cand, double* ms) -> mgs_status {
        mgs_status r;
        *ms = 1e300;
        for (int rep = 0; rep < 5; ++rep) {
            if (rep > 0 && hipEventRecord(e0, stream) != hipSuccess) return fail(ctx, MGS_ERR_HIP, "event");
            if ((r = mgs_forward(f, stream_, g, cams, n_views, &cand, images, nullptr)) != MGS_OK) return r;
            if ((r = mgs_backward(f, stream_, dl_dimages, grads)) != MGS_OK) return r;
            if (rep > 0) {
                float e = 0.f;
                if (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&e, e0, e1) != hipSuccess)
                    return fail(ctx, MGS_ERR_HIP, "event timing");
                *ms = std::min(*ms, (double)e);
            }
        }
        return MGS_OK;
    };
    mgs_settings cur = *base, top = *base;
    double top_ms = 1e300, ms = 0.0;
    mgs_status r = MGS_OK;
    // tile shape x batch depth at two pixels per thread (one for 8x8 tiles)
    const int shapes[4][2] = {{16, 16}, {16, 8}, {32, 8}, {8, 8}};
    const int depths[4] = {32, 64, 128, 256};
    for (int a = 0; a < 4 && r == MGS_OK; ++a) {
        for (int b = 0; b < 4 && r == MGS_OK; ++b) {
            cur = *base;
            cur.tile_w = shapes[a][0];
            cur.tile_h = shapes[a][1];
            cur.batch_depth = depths[b];
            cur.fwd_ppt = cur.bwd_ppt = cur.tile_w * cur.tile_h >= 128 ? 2 : 1;
            if ((r = trial(cur, &ms)) == MGS_OK && ms < top_ms) {
                top_ms = ms;
                top = cur;
            }
        }
    }
    // pixels per thread of each pass and batch depth at the best shape (the
    // best depth depends on the pixels per thread)
    const mgs_settings shape = top;
    for (int b = 0; b < 4 && r == MGS_OK; ++b) {
        for (int fp = 1; fp <= 4 && r == MGS_OK; fp *= 2) {
            for (int bp = 1; bp <= 4 && r == MGS_OK; bp *= 2) {
                cur = shape;
                cur.batch_depth = depths[b];
                cur.fwd_ppt = fp;
                cur.bwd_ppt = bp;
                if (!composite_config_supported(CompositeConfig{cur.tile_w, cur.tile_h, fp}) ||
                    !composite_config_supported(CompositeConfig{cur.tile_w, cur.tile_h, bp}) ||
                    (fp == shape.fwd_ppt && bp == shape.bwd_ppt && cur.batch_depth == shape.batch_depth))
                    continue;
                if ((r = trial(cur, &ms)) == MGS_OK && ms < top_ms) {
                    top_ms = ms;
                    top = cur;
                }
            }
        }
    }
    // wide-list threshold
    const mgs_settings pp = top;
    const int wides[6] = {-1, 8, 16, 32, 64, 256};
    for (int w = 0; w < 6 && r == MGS_OK; ++w) {
        cur = pp;
        cur.wide_tiles = wides[w];
        if (cur.wide_tiles == pp.wide_tiles) continue;
        if ((r = trial(cur, &ms)) == MGS_OK && ms < top_ms) {
            top_ms = ms;
            top = cur;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->prof_on = was_on;
    if (r != MGS_OK) return r;
    *best = top;
    if (best_ms) *best_ms = top_ms;
    return MGS_OK;
}

mgs_status mgs_frame_count_evals(mgs_frame* f, mgs_stream stream_, mgs_eval_counts* out) {
    if (!f || !out) return MGS_ERR_INVALID_ARG;
    mgs_ctx* ctx = f->ctx;
    hipStream_t stream = (hipStream_t)stream_;
    if (!f->have_forward) return fail(ctx, MGS_ERR_STATE, "no forward on this frame");
    if (!f->have_stats) return fail(ctx, MGS_ERR_STATE, "the last forward ran with settings.stats = 0");
    mgs_status s;
    const size_t part = 4 * scan_scratch_bytes(f->P);
    if ((s = grow(ctx, f->sum_tmp, 2 * part + 128))) return s;
    uint64_t* dev = (uint64_t*)((char*)f->sum_tmp.p + 2 * part);
    launch_sum_i32x4(stream, (const int32_t*)f->stats.p, f->P, dev, f->sum_tmp.p);
    launch_sum_i32x4(stream, (const int32_t*)f->evals.p, f->P, dev + 4, (char*)f->sum_tmp.p + part);
    MGS_CHECK_LAUNCH(ctx);
    MGS_HIP(ctx, hipMemcpyAsync(f->h_pinned + 8, dev, 64, hipMemcpyDeviceToHost, stream));
    MGS_HIP(ctx, hipStreamSynchronize(stream));
    out->examined = (int64_t)f->h_pinned[8];
    out->blended = (int64_t)f->h_pinned[9];
    out->blended_masked = (int64_t)f->h_pinned[10];
    out->bwd_examined = (int64_t)f->h_pinned[11];
    out->evaluated = (int64_t)f->h_pinned[12];
    out->bwd_evaluated = (int64_t)f->h_pinned[13];
    return MGS_OK;
}

mgs_status mgs_frame_export(mgs_frame* f, mgs_stream stream, int what, void* dst, size_t* bytes) {
    if (!f || !bytes) return MGS_ERR_INVALID_ARG;
    mgs_ctx* ctx = f->ctx;
    if (!f->have_forward) return fail(ctx, MGS_ERR_STATE, "no forward on this frame");
    const void* src = nullptr;
    size_t n = 0;
    switch (what) {
        case MGS_EXPORT_RECORDS: src = f->rec.p; n = (size_t)f->R * 48; break;
        case MGS_EXPORT_DEPTH: src = f->depth.p; n = (size_t)f->R * 4; break;
        case MGS_EXPORT_RADIUS:
            *bytes = (size_t)f->R * 4;
            if (dst) {
                launch_record_field((hipStream_t)stream, (const float*)f->rec.p, f->R, 7, (float*)dst);
                MGS_CHECK_LAUNCH(ctx);
            }
            return MGS_OK;
        case MGS_EXPORT_TILES: src = f->tiles.p; n = (size_t)f->R * 4; break;
        case MGS_EXPORT_VALUES: src = f->vals_sorted(); n = (size_t)f->K * 4; break;
        case MGS_EXPORT_RANGES: src = f->ranges.p; n = (size_t)(f->total_tiles + f->views.total_regions) * 8; break;
        case MGS_EXPORT_T_FINAL: src = f->t_final.p; n = (size_t)f->P * 4; break;
        case MGS_EXPORT_LAST: src = f->last.p; n = (size_t)f->P * 4; break;
        case MGS_EXPORT_STATS: src = f->stats.p; n = (size_t)f->P * 16; break;
        case MGS_EXPORT_EVALS: src = f->evals.p; n = (size_t)f->P * 16; break;
        case MGS_EXPORT_ORDER: src = f->record_order(); n = (size_t)f->R * 4; break;
        default: return fail(ctx, MGS_ERR_INVALID_ARG, "unknown export %d", what);
    }
    *bytes = n;
    if (dst && n) MGS_HIP(ctx, hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return MGS_OK;
}

mgs_status mgs_profile_enable(mgs_ctx* ctx, int on) {
    if (!ctx) return MGS_ERR_INVALID_ARG;
    for (auto& r : ctx->prof) {
        (void)hipEventSynchronize(r.b);
        ctx->pool.push_back(r.a);
        ctx->pool.push_back(r.b);
    }
    ctx->prof.clear();
    ctx->prof_on = on != 0;
    return MGS_OK;
}

mgs_status mgs_profile_read(mgs_ctx* ctx, double* ms, int64_t* launches) {
    if (!ctx || !ms || !launches) return MGS_ERR_INVALID_ARG;
    for (int i = 0; i < MGS_NUM_STAGES; ++i) {
        ms[i] = 0.0;
        launches[i] = 0;
    }
    for (auto& r : ctx->prof) {
        MGS_HIP(ctx, hipEventSynchronize(r.b));
        float e = 0.f;
        MGS_HIP(ctx, hipEventElapsedTime(&e, r.a, r.b));
        ms[r.stage] += e;
        launches[r.stage] += 1;
        ctx->pool.push_back(r.a);
        ctx->pool.push_back(r.b);
    }
    ctx->prof.clear();
    return MGS_OK;
}

// ---------------------------------------------------------------------------
// stages
// ---------------------------------------------------------------------------

mgs_status mgs_project(mgs_ctx* ctx, mgs_stream stream, const mgs_gaussians* g, const mgs_camera* cams, int n_views,
                       const mgs_settings* st, float* rec, float* depth, float* radius, uint32_t* tiles) {
    if (!ctx) return MGS_ERR_INVALID_ARG;
    mgs_status s;
    if ((s = check_gaussians(ctx, g, true)) || (s = check_cameras(ctx, cams, n_views)) ||
        (s = check_settings(ctx, st)))
        return s;
    if (g->n > 0 && (!rec || !depth || !radius || !tiles)) return fail(ctx, MGS_ERR_INVALID_ARG, "NULL output");
    if (((uintptr_t)rec & 15) != 0) return fail(ctx, MGS_ERR_INVALID_ARG, "rec must be 16-byte aligned");
    ViewSet vs = make_views(cams, n_views, st->tile_w, st->tile_h, nullptr);
    set_limits(vs, cams, st->jac_clamp);
    DevSettings ds = make_settings(st);
    uint32_t* flags = nullptr;
    if (hipMallocAsync((void**)&flags, 16, (hipStream_t)stream) != hipSuccess)
        return fail(ctx, MGS_ERR_OOM, "flag buffer");
    launch_fill_u32((hipStream_t)stream, flags, 4, 0u);
    launch_project_fwd((hipStream_t)stream, *g, vs, ds, rec, depth, radius, tiles, flags);
    (void)hipFreeAsync(flags, (hipStream_t)stream);
    MGS_CHECK_LAUNCH(ctx);
    return MGS_OK;
}

size_t mgs_scan_scratch_bytes(int64_t n) { return scan_scratch_bytes(n < 0 ? 0 : n); }

mgs_status mgs_scan(mgs_ctx* ctx, mgs_stream stream, const uint32_t* in, int64_t n, uint32_t* out,
                    uint64_t* total_dev, void* scratch) {
    if (!ctx) return MGS_ERR_INVALID_ARG;
    if (n < 0) return fail(ctx, MGS_ERR_INVALID_ARG, "n < 0");
    if (n > 0 && (!in || !out || !scratch)) return fail(ctx, MGS_ERR_INVALID_ARG, "NULL argument");
    if (!scratch) return fail(ctx, MGS_ERR_INVALID_ARG, "scratch is NULL");
    launch_scan_u32((hipStream_t)stream, in, n, out, total_dev, scratch);
    MGS_CHECK_LAUNCH(ctx);
    return MGS_OK;
}

mgs_status mgs_scan_noalloc(mgs_ctx* ctx, mgs_stream stream, const uint32_t* in, int64_t n, uint32_t* out,
                            uint64_t* total_dev) {
    if (!ctx) return MGS_ERR_INVALID_ARG;
    if (n < 0) return fail(ctx, MGS_ERR_INVALID_ARG, "n < 0");
    if (n > scan_noalloc_max_n())
        return fail(ctx, MGS_ERR_INVALID_ARG, "n = %lld exceeds the %lld elements the scan's fixed scratch serves",
                    (long long)n, (long long)scan_noalloc_max_n());
    if (n > 0 && (!in || !out)) return fail(ctx, MGS_ERR_INVALID_ARG, "NULL argument");
    if (!ctx->scan_noalloc) return fail(ctx, MGS_ERR_STATE, "no scratch address for device %d", ctx->device);
    launch_scan_u32((hipStream_t)stream, in, n, out, total_dev, ctx->scan_noalloc);
    MGS_CHECK_LAUNCH(ctx);
    return MGS_OK;
}

mgs_status mgs_duplicate(mgs_ctx* ctx, mgs_stream stream, const float* rec, const float* depth, const float* radius,
                         const uint32_t* tiles, const uint32_t* offsets, int64_t n, const mgs_camera* cams,
                         int n_views, const mgs_settings* st, uint64_t* keys, uint32_t* vals, int64_t capacity) {
    if (!ctx) return MGS_ERR_INVALID_ARG;
    mgs_status s;
    if ((s = check_cameras(ctx, cams, n_views)) || (s = check_settings(ctx, st))) return s;
    if (n < 0 || capacity < 0) return fail(ctx, MGS_ERR_INVALID_ARG, "negative size");
    if (n > 0 && (!rec || !depth || !radius || !tiles || !offsets || (capacity > 0 && (!keys || !vals))))
        return fail(ctx, MGS_ERR_INVALID_ARG, "NULL argument");
    ViewSet vs = make_views(cams, n_views, st->tile_w, st->tile_h, nullptr);
    DevSettings ds = make_settings(st);
    uint32_t* flags = nullptr;
    if (hipMallocAsync((void**)&flags, 16, (hipStream_t)stream) != hipSuccess)
        return fail(ctx, MGS_ERR_OOM, "flag buffer");
    launch_fill_u32((hipStream_t)stream, flags, 4, 0u);
    launch_duplicate((hipStream_t)stream, rec, radius, depth, tiles, offsets, n * n_views, n, vs, ds, keys, vals,
                     capacity, flags);
    uint32_t hf = 0;
    MGS_HIP(ctx, hipMemcpyAsync(&hf, flags, 4, hipMemcpyDeviceToHost, (hipStream_t)stream));
    MGS_HIP(ctx, hipStreamSynchronize((hipStream_t)stream));
    (void)hipFreeAsync(flags, (hipStream_t)stream);
    MGS_CHECK_LAUNCH(ctx);
    if (hf & FLAG_CAPACITY) return fail(ctx, MGS_ERR_CAPACITY, "instances exceed capacity %lld", (long long)capacity);
    return MGS_OK;
}

size_t mgs_sort_scratch_bytes(int64_t K) { return sort_scratch_bytes(K < 0 ? 0 : K); }

mgs_status mgs_sort(mgs_ctx* ctx, mgs_stream stream, uint64_t* keys, uint32_t* vals, int64_t K, int key_bits,
                    uint64_t* keys_alt, uint32_t* vals_alt, void* scratch) {
    if (!ctx) return MGS_ERR_INVALID_ARG;
    if (K < 0 || K > (int64_t)0x7fffffff) return fail(ctx, MGS_ERR_INVALID_ARG, "K = %lld", (long long)K);
    if (key_bits < 0 || key_bits > 64) return fail(ctx, MGS_ERR_INVALID_ARG, "key_bits %d", key_bits);
    if (K > 0 && (!keys || !vals || !keys_alt || !vals_alt || !scratch))
        return fail(ctx, MGS_ERR_INVALID_ARG, "NULL argument");
    if (K <= 1) return MGS_OK;
    bool in_alt = false;
    launch_radix_sort((hipStream_t)stream, keys, vals, keys_alt, vals_alt, K, nullptr, key_bits, scratch, &in_alt);
    if (in_alt) {
        MGS_HIP(ctx, hipMemcpyAsync(keys, keys_alt, (size_t)K * 8, hipMemcpyDeviceToDevice, (hipStream_t)stream));
        MGS_HIP(ctx, hipMemcpyAsync(vals, vals_alt, (size_t)K * 4, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    }
    MGS_CHECK_LAUNCH(ctx);
    return MGS_OK;
}

mgs_status mgs_tile_ranges(mgs_ctx* ctx, mgs_stream stream, const uint64_t* keys, int64_t K, int64_t total_tiles,
                           uint32_t* ranges) {
    if (!ctx) return MGS_ERR_INVALID_ARG;
    if (K < 0 || total_tiles < 0) return fail(ctx, MGS_ERR_INVALID_ARG, "negative size");
    if ((K > 0 && !keys) || (total_tiles > 0 && !ranges)) return fail(ctx, MGS_ERR_INVALID_ARG, "NULL argument");
    launch_tile_ranges((hipStream_t)stream, keys, K, nullptr, total_tiles, ranges);
    MGS_CHECK_LAUNCH(ctx);
    return MGS_OK;
}

mgs_status mgs_project_backward(mgs_ctx* ctx, mgs_stream stream, const mgs_gaussians* g, const mgs_camera* cams,
                                int n_views, const mgs_settings* st, const float* d_rec, const mgs_gradients* grads) {
    if (!ctx) return MGS_ERR_INVALID_ARG;
    mgs_status s;
    if ((s = check_settings(ctx, st)) || (s = check_gaussians(ctx, g, st->mask_mode == MGS_MASK_OPACITY)) ||
        (s = check_cameras(ctx, cams, n_views)))
        return s;
    if (!grads || (g->n > 0 && !d_rec)) return fail(ctx, MGS_ERR_INVALID_ARG, "NULL argument");
    if (grads->d_quats && ((uintptr_t)grads->d_quats & 15) != 0)
        return fail(ctx, MGS_ERR_INVALID_ARG, "d_quats must be 16-byte aligned");
    if (grads->accumulate != 0 && grads->accumulate != 1)
        return fail(ctx, MGS_ERR_INVALID_ARG, "accumulate must be 0 or 1");
    ViewSet vs = make_views(cams, n_views, st->tile_w, st->tile_h, nullptr);
    set_limits(vs, cams, st->jac_clamp);
    DevSettings ds = make_settings(st);
    launch_project_bwd((hipStream_t)stream, *g, vs, ds, d_rec, *grads);
    MGS_CHECK_LAUNCH(ctx);
    return MGS_OK;
}

// ---------------------------------------------------------------------------
// masks, loss, optimiser
// ---------------------------------------------------------------------------

mgs_status mgs_sample_masks(mgs_ctx* ctx, mgs_stream stream, const float* scores, int64_t n, float tau, uint64_t seed,
                            uint64_t step, const uint64_t* step_offset, float* m_hard, float* y_soft) {
    if (!ctx) return MGS_ERR_INVALID_ARG;
    if (n < 0) return fail(ctx, MGS_ERR_INVALID_ARG, "n < 0");
    if (!(tau > 0.f)) return fail(ctx, MGS_ERR_INVALID_ARG, "tau must be > 0");
    if (n > 0 && (!scores || !m_hard || !y_soft)) return fail(ctx, MGS_ERR_INVALID_ARG, "NULL argument");
    if (((uintptr_t)scores & 7) != 0) return fail(ctx, MGS_ERR_INVALID_ARG, "scores must be 8-byte aligned");
    StageTimer t(ctx, (hipStream_t)stream, MGS_STAGE_SAMPLE_MASKS);
    launch_sample_masks((hipStream_t)stream, scores, n, tau, seed, step, step_offset, m_hard, y_soft);
    MGS_CHECK_LAUNCH(ctx);
    return MGS_OK;
}

size_t mgs_reduce_scratch_bytes(int64_t n) { return reduce_scratch_bytes(n); }

mgs_status mgs_threshold_masks(mgs_ctx* ctx, mgs_stream stream, const float* scores, int64_t n, float threshold,
                               float* m_hard, float* y_soft) {
    if (!ctx) return MGS_ERR_INVALID_ARG;
    if (n < 0) return fail(ctx, MGS_ERR_INVALID_ARG, "n < 0");
    if (!(threshold > 0.f && threshold < 1.f)) return fail(ctx, MGS_ERR_INVALID_ARG, "threshold must be in (0, 1)");
    if (n > 0 && (!scores || !m_hard || !y_soft)) return fail(ctx, MGS_ERR_INVALID_ARG, "NULL argument");
    if (((uintptr_t)scores & 7) != 0) return fail(ctx, MGS_ERR_INVALID_ARG, "scores must be 8-byte aligned");
    StageTimer t(ctx, (hipStream_t)stream, MGS_STAGE_SAMPLE_MASKS);
    launch_threshold_masks((hipStream_t)stream, scores, n, (double)threshold, m_hard, y_soft);
    MGS_CHECK_LAUNCH(ctx);
    return MGS_OK;
}

mgs_status mgs_prune_sample(mgs_ctx* ctx, mgs_stream stream, const float* scores, int64_t n, uint64_t seed,
                            uint64_t step0, int n_draws, uint32_t* keep) {
    if (!ctx) return MGS_ERR_INVALID_ARG;
    if (n < 0) return fail(ctx, MGS_ERR_INVALID_ARG, "n < 0");
    if (n_draws < 1) return fail(ctx, MGS_ERR_INVALID_ARG, "n_draws must be >= 1");
    if (n > 0 && (!scores || !keep)) return fail(ctx, MGS_ERR_INVALID_ARG, "NULL argument");
    if (((uintptr_t)scores & 7) != 0) return fail(ctx, MGS_ERR_INVALID_ARG, "scores must be 8-byte aligned");
    launch_prune_sample((hipStream_t)stream, scores, n, seed, step0, n_draws, keep);
    MGS_CHECK_LAUNCH(ctx);
    return MGS_OK;
}

size_t mgs_compact_scratch_bytes(int64_t n) {
    return ((size_t)(n > 0 ? n : 1) * 4 + 255) / 256 * 256 + scan_scratch_bytes(n);
}

mgs_status mgs_compact_rows(mgs_ctx* ctx, mgs_stream stream, const uint32_t* keep, int64_t n, int n_arrays,
                            const float* const* in, float* const* out, const int* widths, uint64_t* n_kept,
                            void* scratch) {
    if (!ctx) return MGS_ERR_INVALID_ARG;
    if (n < 0 || n_arrays < 0) return fail(ctx, MGS_ERR_INVALID_ARG, "negative size");
    if (n > (int64_t)0x7fffffff) return fail(ctx, MGS_ERR_INVALID_ARG, "n = %lld exceeds 2^31 - 1", (long long)n);
    if (n_arrays > 0 && (!in || !out || !widths)) return fail(ctx, MGS_ERR_INVALID_ARG, "NULL argument");
    if (n > 0 && (!keep || !scratch)) return fail(ctx, MGS_ERR_INVALID_ARG, "NULL argument");
    for (int a = 0; a < n_arrays; ++a) {
        if (widths[a] < 1 || widths[a] > (1 << 20))
            return fail(ctx, MGS_ERR_INVALID_ARG, "width of array %d must be in 1 .. 2^20", a);
        if (n > 0 && (!in[a] || !out[a])) return fail(ctx, MGS_ERR_INVALID_ARG, "NULL array %d", a);
        if (n > 0 && in[a] == out[a]) return fail(ctx, MGS_ERR_INVALID_ARG, "array %d compacts in place", a);
    }
    hipStream_t st = (hipStream_t)stream;
    uint32_t* pos = reinterpret_cast<uint32_t*>(scratch);
    char* scan_tmp = reinterpret_cast<char*>(scratch) + ((size_t)(n > 0 ? n : 1) * 4 + 255) / 256 * 256;
    if (n > 0) {
        launch_scan_u32(st, keep, n, pos, n_kept, scan_tmp);
        launch_compact_rows(st, keep, pos, n, n_arrays, in, out, widths);
    } else if (n_kept) {
        launch_fill_u32(st, reinterpret_cast<uint32_t*>(n_kept), 2, 0u);
    }
    MGS_CHECK_LAUNCH(ctx);
    return MGS_OK;
}

mgs_status mgs_mask_loss(mgs_ctx* ctx, mgs_stream stream, const float* m_hard, int64_t n, float* loss_m,
                         void* scratch) {
    if (!ctx) return MGS_ERR_INVALID_ARG;
    if (n < 0) return fail(ctx, MGS_ERR_INVALID_ARG, "n < 0");
    if (!loss_m || (n > 0 && (!m_hard || !scratch))) return fail(ctx, MGS_ERR_INVALID_ARG, "NULL argument");
    StageTimer t(ctx, (hipStream_t)stream, MGS_STAGE_MASK_GRAD);
    launch_mask_loss((hipStream_t)stream, m_hard, n, loss_m, scratch);
    MGS_CHECK_LAUNCH(ctx);
    return MGS_OK;
}

mgs_status mgs_mask_grad(mgs_ctx* ctx, mgs_stream stream, const float* d_masks, const float* m_hard,
                         const float* y_soft, int64_t n, float tau, float lambda_m, const float* lambda_scale,
                         float* d_scores, float* loss_m, void* scratch) {
    if (!ctx) return MGS_ERR_INVALID_ARG;
    if (n < 0) return fail(ctx, MGS_ERR_INVALID_ARG, "n < 0");
    if (!(tau > 0.f)) return fail(ctx, MGS_ERR_INVALID_ARG, "tau must be > 0");
    if (n > 0 && (!d_masks || !m_hard || !y_soft || !d_scores || !scratch))
        return fail(ctx, MGS_ERR_INVALID_ARG, "NULL argument");
    if (((uintptr_t)d_scores & 7) != 0) return fail(ctx, MGS_ERR_INVALID_ARG, "d_scores must be 8-byte aligned");
    StageTimer t(ctx, (hipStream_t)stream, MGS_STAGE_MASK_GRAD);
    launch_mask_grad((hipStream_t)stream, d_masks, m_hard, y_soft, n, tau, lambda_m, lambda_scale, d_scores, loss_m,
                     scratch);
    MGS_CHECK_LAUNCH(ctx);
    return MGS_OK;
}

mgs_status mgs_l1_loss_grad(mgs_ctx* ctx, mgs_stream stream, const float* images, const float* targets, int64_t m,
                            float* d_images, const float* grad_scale, float* loss, void* scratch) {
    if (!ctx) return MGS_ERR_INVALID_ARG;
    if (m < 0) return fail(ctx, MGS_ERR_INVALID_ARG, "m < 0");
    if (m > 0 && (!images || !targets || !scratch)) return fail(ctx, MGS_ERR_INVALID_ARG, "NULL argument");
    if (!d_images && !loss) return fail(ctx, MGS_ERR_INVALID_ARG, "neither d_images nor loss requested");
    if (m == 0 && loss) {
        launch_fill_f32((hipStream_t)stream, loss, 1, 0.f);
        MGS_CHECK_LAUNCH(ctx);
        return MGS_OK;
    }
    StageTimer t(ctx, (hipStream_t)stream, MGS_STAGE_LOSS);
    launch_l1_loss_grad((hipStream_t)stream, images, targets, m, d_images, grad_scale, loss, scratch);
    MGS_CHECK_LAUNCH(ctx);
    return MGS_OK;
}

mgs_status mgs_adam_step(mgs_ctx* ctx, mgs_stream stream, float* params, const float* grads, float* m, float* v,
                         int64_t n, float lr, float beta1, float beta2, float eps, int64_t step) {
    if (!ctx) return MGS_ERR_INVALID_ARG;
    if (n < 0 || step < 1) return fail(ctx, MGS_ERR_INVALID_ARG, "n < 0 or step < 1");
    if (n > 0 && (!params || !grads || !m || !v)) return fail(ctx, MGS_ERR_INVALID_ARG, "NULL argument");
    StageTimer t(ctx, (hipStream_t)stream, MGS_STAGE_ADAM);
    launch_adam((hipStream_t)stream, params, grads, m, v, n, lr, beta1, beta2, eps, step);
    MGS_CHECK_LAUNCH(ctx);
    return MGS_OK;
}

mgs_status mgs_adam_step_multi(mgs_ctx* ctx, mgs_stream stream, const mgs_adam_array* arrays, int n_arrays,
                               float beta1, float beta2, float eps, int64_t step, const int64_t* step_offset) {
    if (!ctx) return MGS_ERR_INVALID_ARG;
    if (n_arrays < 0 || (n_arrays > 0 && !arrays)) return fail(ctx, MGS_ERR_INVALID_ARG, "arrays");
    if (!step_offset && step < 1) return fail(ctx, MGS_ERR_INVALID_ARG, "step < 1");
    if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f))
        return fail(ctx, MGS_ERR_INVALID_ARG, "betas must be in [0, 1)");
    std::vector<AdamArray> xs;
    xs.reserve((size_t)n_arrays);
    for (int a = 0; a < n_arrays; ++a) {
        const mgs_adam_array& x = arrays[a];
        if (x.n < 0) return fail(ctx, MGS_ERR_INVALID_ARG, "array %d: n < 0", a);
        if (x.n > 0 && (!x.params || !x.grads || !x.m || !x.v))
            return fail(ctx, MGS_ERR_INVALID_ARG, "array %d: NULL pointer", a);
        if (x.n > ((int64_t)1 << 40)) return fail(ctx, MGS_ERR_INVALID_ARG, "array %d: n beyond 2^40", a);
        xs.push_back(AdamArray{x.params, x.grads, x.m, x.v, x.n, x.lr});
    }
    StageTimer t(ctx, (hipStream_t)stream, MGS_STAGE_ADAM);
    launch_adam_multi((hipStream_t)stream, xs.data(), n_arrays, beta1, beta2, eps, step, step_offset);
    MGS_CHECK_LAUNCH(ctx);
    return MGS_OK;
}

mgs_status mgs_step_advance(mgs_ctx* ctx, mgs_stream stream, int64_t* counter, int64_t delta) {
    if (!ctx) return MGS_ERR_INVALID_ARG;
    if (!counter) return fail(ctx, MGS_ERR_INVALID_ARG, "counter is NULL");
    launch_step_advance((hipStream_t)stream, counter, delta);
    MGS_CHECK_LAUNCH(ctx);
    return MGS_OK;
}

}  // extern "C"
