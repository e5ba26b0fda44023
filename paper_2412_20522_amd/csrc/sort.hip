// Binning and ordering of (tile, Gaussian) instances on gfx950 (Sec. 3.1:
// only Gaussians that intersect a tile take part in that tile, in depth
// order).
//
// Two equivalent orderings are provided:
//  - the literal one: duplicated 64-bit keys (tile << 32 | depth bits) with
//    value = record id, sorted by a stable LSD radix sort over all
//    significant bits (stage entry points mgs_duplicate / mgs_sort);
//  - the one the whole path uses: records are first sorted by their 32-bit
//    depth key (V*N elements), instances are then emitted in that order with
//    32-bit tile ids, and a stable LSD sort over the tile bits alone (one or
//    two passes) yields the same (tile, depth, record) order with a fraction
//    of the memory traffic, since K is often 100x the record count.
//
// The sort is reduce-then-scan (per-block digit histograms, a scan of each
// digit's row of them, then a stable scatter); it has no inter-block spin
// waits, so it needs no forward-progress guarantee between workgroups.
#include <mutex>

#include "common.hpp"
#include "kernels.hpp"

namespace mgs {
namespace {

// Scratch of the allocation-free scan (mgs_scan_noalloc): file-scope device
// memory, one copy per GPU, held until the process ends.  Host code never
// uses this name as an address: the per-device address comes from
// hipGetSymbolAddress (scan_noalloc_init) and is passed to the kernels.
static __device__ __align__(256) unsigned char scratch[SCAN_NOALLOC_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[MAX_DEVICES] = {};

constexpr int NT = 256;
constexpr int IPT = 16;
constexpr int TILE = NT * IPT;  // 4096 elements per block
constexpr int RADIX = 256;
static_assert(NT == RADIX, "one thread per digit in the histogram and scatter steps");
constexpr int64_t SORT_BLOCKS = 2048;  // 8 workgroups per CU on a 256-CU device

template <typename T>
__device__ __forceinline__ T wave_inclusive_scan(T x) {
    const int lane = lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const T y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    return x;
}

// Exclusive scan over a 256-thread block; *total gets the block sum.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* sh, T* total) {
    const T inc = wave_inclusive_scan(v);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 63) sh[w] = inc;
    __syncthreads();
    T wo = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) {
        if (i < w) wo += sh[i];
        tot += sh[i];
    }
    *total = tot;
    __syncthreads();
    return wo + inc - v;
}

// The same over a block of NTH threads (a multiple of 64).
template <typename T, int NTH>
__device__ __forceinline__ T block_exclusive_scan_n(T v, T* sh, T* total) {
    const T inc = wave_inclusive_scan(v);
    const int w = threadIdx.x >> 6;
    if (lane_id() == 63) sh[w] = inc;
    __syncthreads();
    T wo = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NTH / 64; ++i) {
        if (i < w) wo += sh[i];
        tot += sh[i];
    }
    *total = tot;
    __syncthreads();
    return wo + inc - v;
}

__host__ __device__ inline int64_t nblocks(int64_t n) { return (n + TILE - 1) / TILE; }

// Items per thread of the sort's tiles: 8 for 64-bit keys (with 16, the
// keys, values and ranks a thread holds take 188 registers, two waves per
// SIMD), 16 for 32-bit keys.
template <typename KeyT>
constexpr int sort_ipt() {
    return sizeof(KeyT) == 8 ? 8 : 16;
}
template <typename KeyT>
constexpr int sort_tile() {
    return NT * sort_ipt<KeyT>();
}
constexpr int SORT_TILE_MIN = NT * 8;  // the smallest sort tile (sizes the histograms)
constexpr int64_t MAX_SORT_SEGMENTS = 16;  // segments of a segmented sort (one per view)

// Keys per workgroup of the sort: the host's chunk for a known count; with a
// device-side live count, the live keys are spread evenly over the nb
// workgroups the grid was sized for.
template <typename KeyT>
__device__ __forceinline__ int64_t sort_chunk(int64_t K, const uint64_t* K_dev, int64_t nb, int64_t chunk) {
    if (!K_dev) return chunk;
    constexpr int64_t ST = sort_tile<KeyT>();
    return (((K + ST - 1) / ST + nb - 1) / nb) * ST;
}

// ---------------------------------------------------------------------------
// scan of u32 counts (reduce, scan of block sums, downsweep)
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(NT) scan_reduce_kernel(const uint32_t* __restrict__ in, int64_t n,
                                                          uint64_t* __restrict__ partial) {
    __shared__ uint64_t sh[NT / 64];
    const int64_t base = (int64_t)blockIdx.x * TILE;
    uint64_t s = 0;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const int64_t i = base + j * NT + threadIdx.x;
        if (i < n) s += in[i];
    }
    s = wave_inclusive_scan(s);
    if (lane_id() == 63) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t t = 0;
        for (int i = 0; i < NT / 64; ++i) t += sh[i];
        partial[blockIdx.x] = t;
    }
}

__global__ void __launch_bounds__(NT) scan_partials_kernel(uint64_t* __restrict__ partial, int64_t nb,
                                                            uint64_t* __restrict__ total_dev) {
    __shared__ uint64_t sh[NT / 64];
    uint64_t carry = 0;
    for (int64_t base = 0; base < nb; base += NT) {
        const int64_t i = base + threadIdx.x;
        const uint64_t v = i < nb ? partial[i] : 0;
        uint64_t tot;
        const uint64_t ex = block_exclusive_scan(v, sh, &tot);
        if (i < nb) partial[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0 && total_dev) *total_dev = carry;
}

__global__ void __launch_bounds__(NT) scan_down_kernel(const uint32_t* __restrict__ in, int64_t n,
                                                        const uint64_t* __restrict__ partial,
                                                        uint32_t* __restrict__ out) {
    __shared__ uint32_t tile[TILE];
    __shared__ uint32_t sh[NT / 64];
    const int64_t base = (int64_t)blockIdx.x * TILE;
    // coalesced load, then each thread takes 16 consecutive elements
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const int64_t i = base + j * NT + threadIdx.x;
        tile[j * NT + threadIdx.x] = i < n ? in[i] : 0u;
    }
    __syncthreads();
    uint32_t v[IPT];
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        v[j] = tile[threadIdx.x * IPT + j];
        s += v[j];
    }
    uint32_t tot;
    uint32_t run = block_exclusive_scan(s, sh, &tot) + (uint32_t)partial[blockIdx.x];
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        tile[threadIdx.x * IPT + j] = run;
        run += v[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const int64_t i = base + j * NT + threadIdx.x;
        if (i < n) out[i] = tile[j * NT + threadIdx.x];
    }
}

// ---------------------------------------------------------------------------
// literal key duplication (stage API): one thread per record
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(256) duplicate_kernel(
    const float4* __restrict__ rec, const float* __restrict__ radius, const float* __restrict__ depth,
    const uint32_t* __restrict__ tiles, const uint32_t* __restrict__ offsets, int64_t n_records, int64_t n_per_view,
    ViewSet views, DevSettings st, uint64_t* __restrict__ keys, uint32_t* __restrict__ vals, int64_t capacity,
    uint32_t* __restrict__ flags) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_records) return;
    const uint32_t cnt = tiles[r];
    if (cnt == 0) return;
    const int vi = (int)(r / n_per_view);
    const DevView& cam = views.v[vi];
    const Rect q = record_rect(rec, radius, r, cam, st);
    const uint64_t dbits = (uint64_t)__float_as_uint(depth[r]);
    int64_t off = offsets[r];
    bool overflow = false;
    for (int ty = q.y0; ty <= q.y1; ++ty) {
        const uint64_t row = (uint64_t)cam.tile_off + (uint64_t)ty * cam.grid_w;
        for (int tx = q.x0; tx <= q.x1; ++tx) {
            if (off < capacity) {
                keys[off] = ((row + tx) << 32) | dbits;
                vals[off] = (uint32_t)r;
            } else {
                overflow = true;
            }
            ++off;
        }
    }
    if (overflow) atomicOr(flags, FLAG_CAPACITY);
}

// ---------------------------------------------------------------------------
// LSD radix sort, 8 bits per pass, 32- or 64-bit keys with u32 values
// ---------------------------------------------------------------------------

__device__ __forceinline__ int64_t live_count(int64_t K, const uint64_t* K_dev) {
    if (!K_dev) return K;
    const uint64_t k = *K_dev;
    return (int64_t)(k < (uint64_t)K ? k : (uint64_t)K);
}

template <typename KeyT>
__device__ __forceinline__ uint32_t digit_of(KeyT k, int shift) {
    return (uint32_t)(k >> shift) & (RADIX - 1);
}

// Segments: the keys may form consecutive segments of seg_len keys each
// (the last one shorter), sorted each on its own: block b works in segment
// b / nbs, on the (b % nbs)-th chunk of it, and the histograms are laid out
// (segment, digit, block).  A block's output position for digit d is the
// segment's start (seg * seg_len), plus the segment's counts of the digits
// below d, plus the counts of d in the segment's earlier blocks: the
// row scan gives the last term and the row totals, the scatter adds the
// rest.  With one segment (seg_len >= K, nbs = nb) the layout is the plain
// digit-major hist[d * nb + block].
struct SortSeg {
    int64_t seg, bl, beg, end;  // segment, block within it, chunk [beg, end)
};

// Logical block of this workgroup.  Workgroups are dealt to the 8 XCDs in
// turn (workgroup i to XCD i mod 8); the mapping gives every XCD one run of
// consecutive logical blocks, so the digit runs that neighbouring blocks
// scatter next to each other are written through the same L2.
__device__ __forceinline__ int64_t sort_block(int64_t nb) {
    const int64_t i = (int64_t)blockIdx.x;
    const int64_t q = nb >> 3, r = nb & 7, x = i & 7;
    return x * q + (x < r ? x : r) + (i >> 3);
}

__device__ __forceinline__ SortSeg sort_seg(int64_t K, int64_t seg_len, int64_t nbs, int64_t chunk, int64_t nb) {
    SortSeg s;
    const int64_t b = sort_block(nb);
    s.seg = b / nbs;
    s.bl = b - s.seg * nbs;
    const int64_t sbeg = s.seg * seg_len;
    const int64_t send = min(sbeg + seg_len, K);
    s.beg = sbeg + s.bl * chunk;
    s.end = min(s.beg + chunk, send);
    return s;
}

// Per-block digit histograms, written (segment, digit, block)-major.
// Loads are vectorised and coalesced; each lane counts runs of equal digits
// in registers before touching LDS, so keys clustered by digit (neighbouring
// tiles of one splat) do not serialise on one LDS counter.
// Each block owns a contiguous chunk of `chunk` keys (a multiple of the sort tile),
// so a couple of thousand blocks cover any K and the digit-major histogram
// stays small.
// COPIES histograms per wave (lane mod COPIES picks one), so that lanes of
// a wave with equal digits rarely hit one LDS counter: 4 for the list
// entries' cell keys (digits clustered in the second pass), 1 for the
// depth keys
template <typename KeyT, int COPIES>
__global__ void __launch_bounds__(NT) radix_upsweep_kernel(const KeyT* __restrict__ keys, int64_t Kcap,
                                                            const uint64_t* __restrict__ K_dev, int shift,
                                                            uint32_t* __restrict__ hist, int64_t nb, int64_t chunk,
                                                            int64_t seg_len, int64_t nbs) {
    constexpr int VEC = 16 / sizeof(KeyT);  // keys per 16-byte load
    constexpr int SIPT = sort_ipt<KeyT>(), STILE = sort_tile<KeyT>();
    __shared__ uint32_t h[(NT / 64) * COPIES][RADIX];
    const int w = (threadIdx.x >> 6) * COPIES + (lane_id() & (COPIES - 1));
    for (int i = threadIdx.x; i < (NT / 64) * COPIES * RADIX; i += NT) (&h[0][0])[i] = 0u;
    __syncthreads();
    const int64_t K = live_count(Kcap, K_dev);
    chunk = sort_chunk<KeyT>(K, K_dev, nb, chunk);
    const SortSeg sg = sort_seg(K, seg_len, nbs, chunk, nb);
    const int64_t cbeg = sg.beg, cend = sg.end;
    for (int64_t base = cbeg; base < cend; base += STILE)
#pragma unroll
    for (int j = 0; j < SIPT / VEC; ++j) {
        const int64_t i0 = base + ((int64_t)j * NT + threadIdx.x) * VEC;
        KeyT k[VEC];
        int nv = 0;
        if (i0 + VEC <= cend) {
            if constexpr (VEC == 4) {
                const uint4 q = *reinterpret_cast<const uint4*>(keys + i0);
                k[0] = q.x; k[1] = q.y; k[2] = q.z; k[3] = q.w;
            } else {
                const ulonglong2 q = *reinterpret_cast<const ulonglong2*>(keys + i0);
                k[0] = q.x; k[1] = q.y;
            }
            nv = VEC;
        } else {
            for (int v = 0; v < VEC; ++v)
                if (i0 + v < cend) { k[v] = keys[i0 + v]; nv = v + 1; }
        }
        if (nv > 0) {
            uint32_t cur = digit_of(k[0], shift), run = 1;
            for (int v = 1; v < nv; ++v) {
                const uint32_t d = digit_of(k[v], shift);
                if (d == cur) {
                    ++run;
                } else {
                    atomicAdd(&h[w][cur], run);
                    cur = d;
                    run = 1;
                }
            }
            atomicAdd(&h[w][cur], run);
        }
    }
    __syncthreads();
    const int d = threadIdx.x;  // NT == RADIX
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < (NT / 64) * COPIES; ++i) s += h[i][d];
    hist[(sg.seg * RADIX + d) * nbs + sg.bl] = s;
}

// Exclusive prefix of every (segment, digit) row of the block histograms
// over the row's blocks, and the row's total: one workgroup per row, each
// thread over a run of at most SORT_BLOCKS / NT consecutive blocks.
constexpr int ROW_PER_THREAD = (int)(SORT_BLOCKS / NT);
__global__ void __launch_bounds__(NT) radix_rowscan_kernel(const uint32_t* __restrict__ hist, int64_t nbs,
                                                            uint32_t* __restrict__ row_pre,
                                                            uint32_t* __restrict__ row_tot) {
    __shared__ uint32_t sh[NT / 64];
    const int64_t row = blockIdx.x;
    const uint32_t* h = hist + row * nbs;
    uint32_t* p = row_pre + row * nbs;
    const int per = (int)((nbs + NT - 1) / NT);
    const int64_t b0 = (int64_t)threadIdx.x * per;
    uint32_t v[ROW_PER_THREAD];
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < ROW_PER_THREAD; ++j) {
        v[j] = (j < per && b0 + j < nbs) ? h[b0 + j] : 0u;
        s += v[j];
    }
    uint32_t tot;
    uint32_t run = block_exclusive_scan(s, sh, &tot);
#pragma unroll
    for (int j = 0; j < ROW_PER_THREAD; ++j) {
        if (j < per && b0 + j < nbs) p[b0 + j] = run;
        run += v[j];
    }
    if (threadIdx.x == 0) row_tot[row] = tot;
}

// Threads of a scatter workgroup: 512 for 32-bit keys (8 per thread, so
// that twice the waves of a 256-thread workgroup share the tile's LDS), 256
// for 64-bit keys.
template <typename KeyT>
constexpr int sort_dt() {
    return sizeof(KeyT) == 8 ? 256 : 512;
}

// Threads t < RADIX own digit t in the digit steps; the per-wave digit
// counts (at most 64 x 8 per wave, prefixes at most the tile) fit 16 bits.
template <typename KeyT>
__global__ void __launch_bounds__(sort_dt<KeyT>()) __attribute__((amdgpu_waves_per_eu(sizeof(KeyT) == 8 ? 1 : 6)))
radix_downsweep_kernel(
    const KeyT* __restrict__ keys_in, const uint32_t* __restrict__ vals_in, KeyT* __restrict__ keys_out,
    uint32_t* __restrict__ vals_out, int64_t Kcap, const uint64_t* __restrict__ K_dev, int shift,
    const uint32_t* __restrict__ row_pre, const uint32_t* __restrict__ row_tot, int64_t nb, int64_t chunk,
    int64_t seg_len, int64_t nbs) {
    constexpr int DT = sort_dt<KeyT>();
    constexpr int STILE = sort_tile<KeyT>(), SIPT = STILE / DT;
    static_assert(SIPT * 64 <= 65535 && STILE <= 65535, "16-bit digit counts");
    __shared__ KeyT sk[STILE];
    __shared__ uint32_t sv[STILE];
    __shared__ uint16_t wcnt[DT / 64][RADIX];
    __shared__ uint32_t dstart[RADIX];
    __shared__ uint32_t gstart[RADIX];
    __shared__ uint32_t scan_sh[DT / 64];

    const int64_t K = live_count(Kcap, K_dev);
    chunk = sort_chunk<KeyT>(K, K_dev, nb, chunk);
    const SortSeg sg = sort_seg(K, seg_len, nbs, chunk, nb);
    const int64_t cbeg = sg.beg, cend = sg.end;
    if (cbeg >= cend) return;  // uniform over the block
    const int w = threadIdx.x >> 6, lane = lane_id();
    // global start of each digit for this chunk, advanced after every sub-tile
    const bool dig = threadIdx.x < RADIX;
    {
        const int64_t row = sg.seg * RADIX + (dig ? threadIdx.x : 0);
        uint32_t tot;
        const uint32_t below = block_exclusive_scan_n<uint32_t, DT>(dig ? row_tot[row] : 0u, scan_sh, &tot);
        if (dig) gstart[threadIdx.x] = (uint32_t)(sg.seg * seg_len) + below + row_pre[row * nbs + sg.bl];
    }
    for (int64_t base = cbeg; base < cend; base += STILE) {
    const int nvalid = (int)min((int64_t)STILE, cend - base);
    for (int i = threadIdx.x; i < (DT / 64) * RADIX; i += DT) (&wcnt[0][0])[i] = 0u;
    __syncthreads();

    // wave w owns the contiguous span [w * 64 SIPT, (w + 1) * 64 SIPT) of the tile;
    // round j covers 64 consecutive items, lane l the (j * 64 + l)-th
    KeyT key[SIPT];
    uint32_t val[SIPT];
    uint32_t rank[SIPT];
    // one address per array: the rounds are constant offsets from it
    const int l0 = w * (SIPT * 64) + lane;
    const KeyT* kp = keys_in + base + l0;
    const uint32_t* vp = vals_in + base + l0;
#pragma unroll
    for (int j = 0; j < SIPT; ++j) {
        if (l0 + j * 64 < nvalid) {
            key[j] = kp[j * 64];
            val[j] = vp[j * 64];
        } else {
            key[j] = ~(KeyT)0;  // digit 255 at every shift, ranked after every valid item
            val[j] = 0u;
        }
    }
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int j = 0; j < SIPT; ++j) {
        const uint32_t d = digit_of(key[j], shift);
        uint64_t peers = ~0ull;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t bal = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bal : ~bal;
        }
        const uint32_t before = wcnt[w][d];
        rank[j] = before + (uint32_t)__popcll(peers & lt);
        const int leader = __ffsll((long long)peers) - 1;
        if (lane == leader) wcnt[w][d] = (uint16_t)(before + (uint32_t)__popcll(peers));
    }
    // the keys pass through an empty asm statement, so that the scatter below
    // derives each item's digit again instead of keeping its counter address
    // live (in registers) across the digit scan
#pragma unroll
    for (int j = 0; j < SIPT; ++j) asm volatile("" : "+v"(key[j]));
    __syncthreads();
    // per digit: offsets of each wave, block total, then block-wide digit starts
    uint32_t digit_total = 0;
    {
        const int d = threadIdx.x;
        uint32_t run = 0;
        if (dig) {
#pragma unroll
            for (int i = 0; i < DT / 64; ++i) {
                const uint32_t c = wcnt[i][d];
                wcnt[i][d] = (uint16_t)run;
                run += c;
            }
        }
        uint32_t tot;
        const uint32_t ds = block_exclusive_scan_n<uint32_t, DT>(run, scan_sh, &tot);
        if (dig) dstart[d] = ds;
        digit_total = run;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < SIPT; ++j) {
        const uint32_t d = digit_of(key[j], shift);
        const uint32_t pos = dstart[d] + wcnt[w][d] + rank[j];
        sk[pos] = key[j];
        sv[pos] = val[j];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nvalid; i += DT) {
        const KeyT k = sk[i];
        const uint32_t d = digit_of(k, shift);
        const uint32_t o = gstart[d] + (uint32_t)i - dstart[d];
        keys_out[o] = k;
        vals_out[o] = sv[i];
    }
    __syncthreads();
    // padded items all carry digit 255 and sit past nvalid; they are not counted
    const uint32_t pad = (threadIdx.x == RADIX - 1) ? (uint32_t)(STILE - nvalid) : 0u;
    if (dig) gstart[threadIdx.x] += digit_total - pad;
    __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// tile ranges, fills, sums
// ---------------------------------------------------------------------------

// [start, end) of every bin of sorted keys; keys at or past nbins (entries
// that belong nowhere, sorted last) are left out of every range.
template <typename KeyT>
__global__ void __launch_bounds__(256) tile_ranges_kernel(const KeyT* __restrict__ keys, int64_t Kcap,
                                                           const uint64_t* __restrict__ K_dev, int shift,
                                                           uint64_t nbins, uint2* __restrict__ ranges) {
    const int64_t K = live_count(Kcap, K_dev);
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    const uint64_t t = (uint64_t)(keys[k] >> shift);
    const bool tv = t < nbins;
    if (k == 0) {
        if (tv) ranges[t].x = 0;
    } else {
        const uint64_t p = (uint64_t)(keys[k - 1] >> shift);
        if (p != t) {
            if (p < nbins) ranges[p].y = (uint32_t)k;
            if (tv) ranges[t].x = (uint32_t)k;
        }
    }
    if (k == K - 1 && tv) ranges[t].y = (uint32_t)K;
}

// The same for 32-bit keys, four consecutive keys per thread (one 16-byte
// load of keys 4 j .. 4 j + 3 and the key before them).
__global__ void __launch_bounds__(256) tile_ranges4_kernel(const uint32_t* __restrict__ keys, int64_t Kcap,
                                                            const uint64_t* __restrict__ K_dev, uint64_t nbins,
                                                            uint2* __restrict__ ranges) {
    const int64_t K = live_count(Kcap, K_dev);
    const int64_t k0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (k0 >= K) return;
    uint32_t v[4];
    if (k0 + 4 <= K) {
        const uint4 q = *reinterpret_cast<const uint4*>(keys + k0);
        v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = k0 + i < K ? keys[k0 + i] : 0u;
    }
    uint64_t p = k0 > 0 ? (uint64_t)keys[k0 - 1] : 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t k = k0 + i;
        if (k >= K) break;
        const uint64_t t = v[i];
        const bool tv = t < nbins;
        if (k == 0) {
            if (tv) ranges[t].x = 0;
        } else if (p != t) {
            if (p < nbins) ranges[p].y = (uint32_t)k;
            if (tv) ranges[t].x = (uint32_t)k;
        }
        if (k == K - 1 && tv) ranges[t].y = (uint32_t)K;
        p = t;
    }
}

__global__ void __launch_bounds__(256) fill_u32_kernel(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Up to FILL_SPANS u32 spans in one launch: element i of the concatenation
// belongs to the first span whose end exceeds it.
struct FillSet {
    uint32_t* p[FILL_SPANS];
    int64_t end[FILL_SPANS];  // cumulative element counts
    uint32_t v[FILL_SPANS];
    int count;
};

__global__ void __launch_bounds__(256) fill_set_kernel(FillSet fs) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t start = 0;
    for (int k = 0; k < fs.count; ++k) {
        if (i < fs.end[k]) {
            fs.p[k][i - start] = fs.v[k];
            return;
        }
        start = fs.end[k];
    }
}

__global__ void __launch_bounds__(256) fill_f32_kernel(float* __restrict__ p, int64_t n, float v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void __launch_bounds__(256) round_f64_kernel(const double* __restrict__ in, float* __restrict__ out,
                                                         int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}

__global__ void __launch_bounds__(NT) sum_i32x4_partial_kernel(const int4* __restrict__ in, int64_t n,
                                                                uint64_t* __restrict__ partial, int64_t nb) {
    __shared__ uint64_t sh[4][NT / 64];
    const int64_t base = (int64_t)blockIdx.x * TILE;
    uint64_t s[4] = {0, 0, 0, 0};
    for (int j = 0; j < IPT; ++j) {
        const int64_t i = base + j * NT + threadIdx.x;
        if (i < n) {
            const int4 v = in[i];
            s[0] += (uint64_t)(int64_t)v.x;
            s[1] += (uint64_t)(int64_t)v.y;
            s[2] += (uint64_t)(int64_t)v.z;
            s[3] += (uint64_t)(int64_t)v.w;
        }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const uint64_t x = wave_inclusive_scan(s[c]);
        if (lane_id() == 63) sh[c][threadIdx.x >> 6] = x;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        uint64_t t = 0;
        for (int i = 0; i < NT / 64; ++i) t += sh[threadIdx.x][i];
        partial[threadIdx.x * nb + blockIdx.x] = t;
    }
}

// seg_len > 0: the keys form segments of seg_len keys, each sorted on its own
// (no device-side count then); otherwise one segment.
template <typename KeyT>
void radix_sort_t(hipStream_t stream, KeyT* keys, uint32_t* vals, KeyT* keys_alt, uint32_t* vals_alt, int64_t K,
                  const uint64_t* K_dev, int begin_bit, int end_bit, void* scratch, bool* out_in_alt,
                  int64_t seg_len = 0) {
    *out_in_alt = false;
    if (K <= 1 && !K_dev) return;
    if (end_bit <= begin_bit) return;
    // about SORT_BLOCKS workgroups, each over a contiguous chunk of whole
    // tiles of one segment
    constexpr int64_t STILE = sort_tile<KeyT>();
    const bool segmented = seg_len > 0 && seg_len < K && !K_dev;
    const int64_t slen = segmented ? seg_len : (K > 0 ? K : 1);
    const int64_t nseg = segmented ? (K + seg_len - 1) / seg_len : 1;
    const int64_t per_seg = std::max<int64_t>(1, SORT_BLOCKS / nseg);
    const int64_t ntiles = (slen + STILE - 1) / STILE;
    const int64_t tiles_per_block = (ntiles + per_seg - 1) / per_seg;
    const int64_t chunk = tiles_per_block * STILE;
    const int64_t nbs = (ntiles + tiles_per_block - 1) / tiles_per_block;
    const int64_t nb = nseg * nbs;
    const int64_t seg_arg = segmented ? seg_len : INT64_MAX / 4;
    static_assert(SORT_BLOCKS % NT == 0, "row scan: whole runs per thread");
    const int64_t hn = nb * RADIX, rows = nseg * RADIX;
    uint32_t* hist = reinterpret_cast<uint32_t*>(scratch);
    uint32_t* row_pre = hist + hn;
    uint32_t* row_tot = row_pre + hn;
    KeyT* kin = keys;
    uint32_t* vin = vals;
    KeyT* kout = keys_alt;
    uint32_t* vout = vals_alt;
    for (int shift = begin_bit; shift < end_bit; shift += 8) {
        if (segmented)
            hipLaunchKernelGGL((radix_upsweep_kernel<KeyT, 1>), dim3((unsigned)nb), dim3(NT), 0, stream, kin, K, K_dev,
                               shift, hist, nb, chunk, seg_arg, nbs);
        else
            hipLaunchKernelGGL((radix_upsweep_kernel<KeyT, 4>), dim3((unsigned)nb), dim3(NT), 0, stream, kin, K, K_dev,
                               shift, hist, nb, chunk, seg_arg, nbs);
        hipLaunchKernelGGL(radix_rowscan_kernel, dim3((unsigned)rows), dim3(NT), 0, stream, (const uint32_t*)hist,
                           nbs, row_pre, row_tot);
        hipLaunchKernelGGL(radix_downsweep_kernel<KeyT>, dim3((unsigned)nb), dim3(sort_dt<KeyT>()), 0, stream, kin, vin,
                           kout, vout,
                           K, K_dev, shift, (const uint32_t*)row_pre, (const uint32_t*)row_tot, nb, chunk, seg_arg,
                           nbs);
        KeyT* tk = kin; kin = kout; kout = tk;
        uint32_t* tv = vin; vin = vout; vout = tv;
        *out_in_alt = !*out_in_alt;
    }
}

}  // namespace

size_t scan_scratch_bytes(int64_t n) { return (size_t)(nblocks(n) + 1) * sizeof(uint64_t) + 256; }

int64_t scan_noalloc_max_n() {
    // the scan needs (blocks + 1) u64 partial sums plus 256 bytes
    const int64_t blocks = (int64_t)((SCAN_NOALLOC_BYTES - 256) / sizeof(uint64_t)) - 1;
    return blocks * TILE;
}

hipError_t scan_noalloc_init(int device, void** out) {
    *out = nullptr;
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[device]) {
        // with `device` current: its own copy of the array
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_noalloc_ptr[device] = p;
    }
    *out = g_noalloc_ptr[device];
    return hipSuccess;
}

void launch_scan_u32(hipStream_t stream, const uint32_t* in, int64_t n, uint32_t* out, uint64_t* total_dev,
                     void* scratch) {
    const int64_t nb = nblocks(n);
    uint64_t* partial = reinterpret_cast<uint64_t*>(scratch);
    if (n == 0) {
        if (total_dev) hipLaunchKernelGGL(scan_partials_kernel, dim3(1), dim3(NT), 0, stream, partial, (int64_t)0,
                                          total_dev);
        return;
    }
    hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)nb), dim3(NT), 0, stream, in, n, partial);
    hipLaunchKernelGGL(scan_partials_kernel, dim3(1), dim3(NT), 0, stream, partial, nb, total_dev);
    hipLaunchKernelGGL(scan_down_kernel, dim3((unsigned)nb), dim3(NT), 0, stream, in, n,
                       (const uint64_t*)partial, out);
}

void launch_duplicate(hipStream_t stream, const float* rec, const float* radius, const float* depth,
                      const uint32_t* tiles, const uint32_t* offsets, int64_t n_records, int64_t n_per_view,
                      const ViewSet& views, const DevSettings& st, uint64_t* keys, uint32_t* vals, int64_t capacity,
                      uint32_t* flags) {
    if (n_records == 0) return;
    hipLaunchKernelGGL(duplicate_kernel, dim3((unsigned)((n_records + 255) / 256)), dim3(256), 0, stream,
                       reinterpret_cast<const float4*>(rec), radius, depth, tiles, offsets, n_records, n_per_view,
                       views, st, keys, vals, capacity, flags);
}

size_t sort_scratch_bytes(int64_t K) {
    // workgroups of a sort of K keys: at most one per tile of the smallest
    // tile size plus one per segment (at most MAX_SORT_SEGMENTS), and at
    // most SORT_BLOCKS (the launcher's bound)
    const int64_t nb = std::min<int64_t>(((K > 0 ? K : 1) + SORT_TILE_MIN - 1) / SORT_TILE_MIN + MAX_SORT_SEGMENTS,
                                         SORT_BLOCKS);
    const int64_t hist = nb * RADIX;
    return (size_t)(2 * hist + MAX_SORT_SEGMENTS * RADIX) * sizeof(uint32_t) + 1024;
}

void launch_radix_sort(hipStream_t stream, uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt,
                       int64_t K, const uint64_t* K_dev, int key_bits, void* scratch, bool* out_in_alt) {
    radix_sort_t<uint64_t>(stream, keys, vals, keys_alt, vals_alt, K, K_dev, 0, key_bits, scratch, out_in_alt);
}

void launch_radix_sort32(hipStream_t stream, uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                         int64_t K, const uint64_t* K_dev, int begin_bit, int end_bit, void* scratch,
                         bool* out_in_alt) {
    radix_sort_t<uint32_t>(stream, keys, vals, keys_alt, vals_alt, K, K_dev, begin_bit, end_bit, scratch, out_in_alt);
}

void launch_radix_sort_segmented(hipStream_t stream, uint32_t* keys, uint32_t* vals, uint32_t* keys_alt,
                                 uint32_t* vals_alt, int64_t K, int64_t seg_len, void* scratch, bool* out_in_alt) {
    if (seg_len > 0 && (K + seg_len - 1) / seg_len > MAX_SORT_SEGMENTS) seg_len = 0;  // not reached: views <= 16
    radix_sort_t<uint32_t>(stream, keys, vals, keys_alt, vals_alt, K, nullptr, 0, 32, scratch, out_in_alt, seg_len);
}

void launch_tile_ranges(hipStream_t stream, const uint64_t* keys, int64_t K, const uint64_t* K_dev,
                        int64_t total_tiles, uint32_t* ranges) {
    launch_fill_u32(stream, ranges, 2 * total_tiles, 0u);
    if (K == 0) return;
    hipLaunchKernelGGL(tile_ranges_kernel<uint64_t>, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, stream, keys, K,
                       K_dev, 32, (uint64_t)total_tiles, reinterpret_cast<uint2*>(ranges));
}

void launch_tile_ranges32(hipStream_t stream, const uint32_t* keys, int64_t K, const uint64_t* K_dev,
                          int64_t total_tiles, uint32_t* ranges, bool cleared) {
    if (!cleared) launch_fill_u32(stream, ranges, 2 * total_tiles, 0u);
    if (K == 0) return;
    // keys come from the library's own buffers (16-byte aligned)
    hipLaunchKernelGGL(tile_ranges4_kernel, dim3((unsigned)((K + 1023) / 1024)), dim3(256), 0, stream, keys, K, K_dev,
                       (uint64_t)total_tiles, reinterpret_cast<uint2*>(ranges));
}

void launch_fill_u32(hipStream_t stream, uint32_t* p, int64_t n, uint32_t value) {
    if (n <= 0) return;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, p, n, value);
}

void launch_fill_spans(hipStream_t stream, const FillSpan* spans, int count) {
    FillSet fs{};
    int64_t total = 0;
    for (int k = 0; k < count && fs.count < FILL_SPANS; ++k) {
        if (!spans[k].p || spans[k].n <= 0) continue;
        total += spans[k].n;
        fs.p[fs.count] = spans[k].p;
        fs.end[fs.count] = total;
        fs.v[fs.count] = spans[k].value;
        ++fs.count;
    }
    if (total == 0) return;
    hipLaunchKernelGGL(fill_set_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, stream, fs);
}

void launch_round_f64(hipStream_t stream, const double* in, float* out, int64_t n) {
    if (n <= 0) return;
    hipLaunchKernelGGL(round_f64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, in, out, n);
}

void launch_fill_f32(hipStream_t stream, float* p, int64_t n, float value) {
    if (n <= 0) return;
    hipLaunchKernelGGL(fill_f32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, p, n, value);
}

void launch_sum_i32x4(hipStream_t stream, const int32_t* in, int64_t n, uint64_t* out_dev, void* scratch) {
    const int64_t nb = nblocks(n > 0 ? n : 1);
    uint64_t* partial = reinterpret_cast<uint64_t*>(scratch);
    hipLaunchKernelGGL(sum_i32x4_partial_kernel, dim3((unsigned)nb), dim3(NT), 0, stream,
                       reinterpret_cast<const int4*>(in), n, partial, nb);
    for (int c = 0; c < 4; ++c)
        hipLaunchKernelGGL(scan_partials_kernel, dim3(1), dim3(NT), 0, stream, partial + c * nb, nb, out_dev + c);
}

}  // namespace mgs
