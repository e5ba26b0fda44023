// Host-side launchers of the gfx950 kernels (one translation unit each).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "common.hpp"

namespace mgs {

// projection (radius optional: the record's B.w holds it too)
// rkeys, rvals (optional, both or neither): the keys of the per-view depth
// order of the records (depth bits, all ones for records without tiles) and
// the record ids
void launch_project_fwd(hipStream_t stream, const mgs_gaussians& g, const ViewSet& views, const DevSettings& st,
                        float* rec, float* depth, float* radius, uint32_t* tiles, uint32_t* flags,
                        uint32_t* rkeys = nullptr, uint32_t* rvals = nullptr);
// out[r] = field `field` (0..11) of record r (the radius is field 7, B.w)
void launch_record_field(hipStream_t stream, const float* rec, int64_t R, int field, float* out);
void launch_project_bwd(hipStream_t stream, const mgs_gaussians& g, const ViewSet& views, const DevSettings& st,
                        const float* d_rec, const mgs_gradients& out);
// Whole path: FP64 per-record gradients (zeroed by the forward compositing
// before the backward accumulates them); dm_acc (FP64 mask gradients) is
// rounded into out.d_masks.
void launch_project_bwd64(hipStream_t stream, const mgs_gaussians& g, const ViewSet& views, const DevSettings& st,
                          double* d_rec, const double* dm_acc, const mgs_gradients& out,
                          const uint32_t* tiles);

// scan / binning / sort / ranges
size_t scan_scratch_bytes(int64_t n);
// Exclusive scan of n u32; total (u64) to total_dev.  count_dev (optional)
// holds the live element count on the device (<= n); elements at or past it
// are treated as zero.
void launch_scan_u32(hipStream_t stream, const uint32_t* in, int64_t n, uint32_t* out, uint64_t* total_dev,
                     void* scratch);
// The allocation-free scan: a library-owned device array of
// SCAN_NOALLOC_BYTES per GPU holds its scratch.  scan_noalloc_init, called
// with `device` current, returns that GPU's address of the array (looked up
// once per device); scan_noalloc_max_n is the largest n it serves.
constexpr size_t SCAN_NOALLOC_BYTES = MGS_SCAN_NOALLOC_BYTES;
hipError_t scan_noalloc_init(int device, void** out);
int64_t scan_noalloc_max_n();
void launch_duplicate(hipStream_t stream, const float* rec, const float* radius, const float* depth,
                      const uint32_t* tiles, const uint32_t* offsets, int64_t n_records, int64_t n_per_view,
                      const ViewSet& views, const DevSettings& st, uint64_t* keys, uint32_t* vals, int64_t capacity,
                      uint32_t* flags);
size_t sort_scratch_bytes(int64_t K);
// Sorts (keys, vals) by the low key_bits bits; K_dev (optional) is the live
// count on the device (<= K).  Returns through *out_in_alt whether the
// result ended in the alternate buffers.
void launch_radix_sort(hipStream_t stream, uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt,
                       int64_t K, const uint64_t* K_dev, int key_bits, void* scratch, bool* out_in_alt);
void launch_tile_ranges(hipStream_t stream, const uint64_t* keys, int64_t K, const uint64_t* K_dev,
                        int64_t total_tiles, uint32_t* ranges);
// 32-bit keys sorted on bits [begin_bit, end_bit) (stable), and the tile
// ranges of 32-bit tile keys
void launch_radix_sort32(hipStream_t stream, uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                         int64_t K, const uint64_t* K_dev, int begin_bit, int end_bit, void* scratch,
                         bool* out_in_alt);
// Stable sort of 32-bit keys (all bits) within consecutive segments of
// seg_len keys each (at most 16 segments; the last may be shorter).
void launch_radix_sort_segmented(hipStream_t stream, uint32_t* keys, uint32_t* vals, uint32_t* keys_alt,
                                 uint32_t* vals_alt, int64_t K, int64_t seg_len, void* scratch, bool* out_in_alt);
// cleared: ranges is already zero (else cleared here)
void launch_tile_ranges32(hipStream_t stream, const uint32_t* keys, int64_t K, const uint64_t* K_dev,
                          int64_t total_tiles, uint32_t* ranges, bool cleared = false);
void launch_fill_u32(hipStream_t stream, uint32_t* p, int64_t n, uint32_t value);
// Several u32 fills in one launch (at most FILL_SPANS; null or empty spans
// are skipped).
constexpr int FILL_SPANS = 4;
struct FillSpan {
    uint32_t* p;
    int64_t n;
    uint32_t value;
};
void launch_fill_spans(hipStream_t stream, const FillSpan* spans, int count);
void launch_fill_f32(hipStream_t stream, float* p, int64_t n, float value);
// Column sums of an [n, 4] int32 array into out_dev[4] (u64); scratch holds
// 4 * scan_scratch_bytes(n) bytes.
void launch_sum_i32x4(hipStream_t stream, const int32_t* in, int64_t n, uint64_t* out_dev, void* scratch);

// compositing
struct CompositeConfig {
    int tile_w, tile_h, ppt;  // pixels per thread; threads per block = tile_w * tile_h / ppt
};
bool composite_config_supported(const CompositeConfig& c);

// hybrid binning: records in (view, depth, record) order are copied once
// ("sorted records": radius in B.w, record id bits in C.w); narrow records
// are listed per tile, wide records per region (one key space: tile ids, then
// region ids), with sorted positions as values, and merged per tile while
// compositing
// part: classify_parts_bytes(R) bytes of per-workgroup counts (written by
// the classification) and list offsets (by launch_list_offsets, read by the
// duplication)
size_t classify_parts_bytes(int64_t R);
void launch_permute_classify(hipStream_t stream, const uint32_t* order, const uint32_t* skeys, const float* rec,
                             int64_t R, int64_t n, const ViewSet& views, const DevSettings& st, uint32_t* cnt,
                             uint64_t* tmask, float* srec, uint32_t* part);
// From the classification's per-workgroup counts: each workgroup's first list
// entry, the entry total (device u64 *total) and wide_counts (device u64):
// [0] = wide records, [2] = their region entries
void launch_list_offsets(hipStream_t stream, uint32_t* part, int64_t R, uint64_t* total, uint64_t* wide_counts);
void launch_duplicate_lists(hipStream_t stream, const float* srec, const uint32_t* cnt_sorted,
                            const uint64_t* tmask, uint32_t* part, int64_t R,
                            int64_t n, const ViewSet& views, const DevSettings& st, uint32_t* keys, uint32_t* vals,
                            int64_t capacity, uint32_t* flags);
// Tile order of a persistent launch: the tiles by descending cost key
// (key[t] in 0..255, ties in any order), so that the most expensive start
// first.  hist_cursor: [512] u32 of scratch (cleared here unless cleared).
void launch_tile_order(hipStream_t stream, const uint32_t* key, uint32_t tiles, uint32_t* hist_cursor,
                       uint32_t* order, bool cleared = false);
// The forward's per-tile set-up after the ranges: each tile's first batch
// checkpoint (cur_off, and the total into the device u64 *cur_need: per tile
// 2 (ceil(narrow / batch) + ceil(region / batch)) + 2), its cost key (cost:
// the entries of its two lists in units of 8, at most 255), and the tile
// order by descending key (key[t], or the cost key when key is null).
// hist_cursor: [512] u32, zero before; blk: blocks of 256 tiles, u32 scratch.
void launch_tile_setup(hipStream_t stream, const uint32_t* ranges, const ViewSet& views, int batch,
                       const uint32_t* key, uint32_t* cost, uint32_t* cur_off, uint64_t* cur_need, uint32_t* blk,
                       uint32_t* hist_cursor, uint32_t* order);
struct HybridBuffers {
    const uint32_t* vals;        // list entries (sorted positions), (cell, position) order
    const uint32_t* ranges;      // [tiles + regions, 2]
    uint32_t* cur;               // [checkpoints, 4]
    const uint32_t* cur_off;     // [tiles]
    uint32_t* nbatch;            // [tiles]
    const uint64_t* cur_need;    // device: checkpoints the tiles may take
    uint64_t cur_cap;            // checkpoints the buffer holds
    uint32_t* flags;             // device flags (capacity)
    uint32_t* cur_stg;           // [checkpoints, 2] staged-list offset (or ~0) and count
    uint32_t* stg;               // [stg_cap, 2] staged entries; null: the backward merges again
    uint32_t* stg_count;         // device counter of staged entries (zeroed before the forward)
    uint64_t stg_cap;
    double* drec_clear;          // optional: FP64 per-record gradient accumulator the forward clears
    uint64_t drec_clear_n2;      // its size in pairs of doubles
    const uint32_t* order;       // optional [tiles]: the order in which a persistent launch takes the tiles
};
// stats [P, 4] (examined, blended, blended with mask 0, last + 1) and evals
// [P, 4] (evaluated, evaluated up to the last blended entry, 0, 0) are
// written only when both are non-null.
// imp_sum (FP64, zeroed) and imp_max (float bits, zeroed), both [n] or both
// null: per-Gaussian sum and maximum of the blending weights M alpha T.
void launch_hybrid_fwd(hipStream_t stream, const CompositeConfig& cfg, const float* srec, const HybridBuffers& bufs,
                       const ViewSet& views, const DevSettings& st, float* images, float* t_final, int32_t* last,
                       int32_t* stats, int32_t* evals, uint32_t* queue, int num_cus, int64_t n = 0,
                       double* imp_sum = nullptr, uint32_t* imp_max = nullptr);
void launch_round_f64(hipStream_t stream, const double* in, float* out, int64_t n);
void launch_hybrid_bwd(hipStream_t stream, const CompositeConfig& cfg, const float* srec, const HybridBuffers& bufs,
                       const ViewSet& views, const DevSettings& st, const float* t_final, const int32_t* last,
                       const float* dl_dimages, int64_t n, double* d_rec, double* d_masks, uint32_t* queue,
                       int num_cus);

// masks, loss, optimiser
size_t reduce_scratch_bytes(int64_t n);
// step_off (optional, device): added to step
void launch_sample_masks(hipStream_t stream, const float* scores, int64_t n, float tau, uint64_t seed, uint64_t step,
                         const uint64_t* step_off, float* m_hard, float* y_soft);
void launch_threshold_masks(hipStream_t stream, const float* scores, int64_t n, double threshold, float* m_hard,
                            float* y_soft);
void launch_prune_sample(hipStream_t stream, const float* scores, int64_t n, uint64_t seed, uint64_t step0,
                         int n_draws, uint32_t* keep);
// pos: exclusive scan of keep
void launch_compact_rows(hipStream_t stream, const uint32_t* keep, const uint32_t* pos, int64_t n, int n_arrays,
                         const float* const* in, float* const* out, const int* widths);
void launch_mask_loss(hipStream_t stream, const float* m_hard, int64_t n, float* loss_m, void* scratch);
// lambda_scale (optional, device): multiplies lambda_m
void launch_mask_grad(hipStream_t stream, const float* d_masks, const float* m_hard, const float* y_soft, int64_t n,
                      float tau, float lambda_m, const float* lambda_scale, float* d_scores, float* loss_m,
                      void* scratch);
// d_images and loss optional; grad_scale (optional, device) multiplies d_images
void launch_l1_loss_grad(hipStream_t stream, const float* images, const float* targets, int64_t m, float* d_images,
                         const float* grad_scale, float* loss, void* scratch);
struct AdamArray {
    float* params;
    const float* grads;
    float* m;
    float* v;
    int64_t n;
    float lr;
};
int adam_multi_max();
// step_off (optional, device): added to step for the bias corrections
void launch_adam_multi(hipStream_t stream, const AdamArray* arrays, int n_arrays, float b1, float b2, float eps,
                       int64_t step, const int64_t* step_off);
void launch_step_advance(hipStream_t stream, int64_t* counter, int64_t delta);
void launch_adam(hipStream_t stream, float* params, const float* grads, float* m, float* v, int64_t n, float lr,
                 float b1, float b2, float eps, int64_t step);

}  // namespace mgs
