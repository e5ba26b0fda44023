// Mask sampling and mask gradient (Sec. 3.3, Eq. 7-8), probabilistic
// pruning and row compaction (Sec. 3.5), L1 rendering loss and Adam on
// gfx950.
//
// Masks: two scores per Gaussian, Gumbel-Softmax with a hard forward value
// and the soft sample's derivative in the backward (straight-through).  The
// Gumbel noise is a function of (seed, step, Gaussian id) through
// Philox4x32-10 (Salmon et al., SC'11), so a step can be replayed.  The noise
// and the hard decision are computed in double precision.
#include "common.hpp"
#include "kernels.hpp"

namespace mgs {
namespace {

constexpr int RNT = 256;

// Philox4x32-10: ten rounds of two 32x32->64 multiplies with the Weyl key
// schedule, written from the generator's published definition.
__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3, uint32_t k0,
                                              uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
}

__device__ __forceinline__ double u01_from_bits(uint32_t x) {
    return ((double)(x >> 8) + 0.5) * (1.0 / 16777216.0);
}

__device__ __forceinline__ double gumbel_from_bits(uint32_t x) {
    return -log(-log(u01_from_bits(x)));
}

__global__ void __launch_bounds__(RNT) sample_masks_kernel(const float* __restrict__ scores, int64_t n, float tau,
                                                            uint64_t seed, uint64_t step0,
                                                            const uint64_t* __restrict__ step_off,
                                                            float* __restrict__ m_hard, float* __restrict__ y_soft) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // a step counter kept on the device lets a captured training step draw
    // fresh masks at every replay
    const uint64_t step = step0 + (step_off ? *step_off : 0ull);
    uint32_t c0 = (uint32_t)i, c1 = (uint32_t)((uint64_t)i >> 32), c2 = (uint32_t)step, c3 = (uint32_t)(step >> 32);
    philox4x32_10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
    const float2 s = reinterpret_cast<const float2*>(scores)[i];
    const double z0 = (double)s.x + gumbel_from_bits(c0);
    const double z1 = (double)s.y + gumbel_from_bits(c1);
    m_hard[i] = z0 > z1 ? 1.f : 0.f;
    y_soft[i] = (float)(1.0 / (1.0 + exp(-(z0 - z1) / (double)tau)));
}

// Deterministic masks with a straight-through estimator (the alternative to
// Gumbel sampling in the ablation of Sec. 4.3): y = sigmoid(s0 - s1) and
// M = 1 iff y > threshold, both in double precision.  y_soft = y, so the mask
// gradient with tau = 1 is the straight-through one, dL/dy = dL/dM.
__global__ void __launch_bounds__(RNT) threshold_masks_kernel(const float* __restrict__ scores, int64_t n,
                                                               double threshold, float* __restrict__ m_hard,
                                                               float* __restrict__ y_soft) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float2 s = reinterpret_cast<const float2*>(scores)[i];
    const double y = 1.0 / (1.0 + exp((double)s.y - (double)s.x));
    m_hard[i] = y > threshold ? 1.f : 0.f;
    y_soft[i] = (float)y;
}

// Probabilistic pruning (Sec. 3.5): n_draws hard masks per Gaussian with the
// rule above (steps step0 .. step0 + n_draws - 1); keep[i] = 1 iff any is 1.
// Most draws are decided without the four logarithms: g(u) = -log(-log u)
// increases with u and is at least G_MIN = g(2^-25) over the uniforms the
// generator yields, so with d = s0 - s1 a draw is 0 whatever u1 once
// g(u0) < G_MIN - d, and 1 whatever u0 once g(u1) < G_MIN + d.  Both tests
// compare u with the inverse image of the bound, less 1e-6: the exact gap
// between the two sides is then at least e 1e-6 (g' >= e), far above the
// rounding of the double-precision rule, which therefore decides the same
// way.  The remaining draws take that rule itself.
__global__ void __launch_bounds__(RNT) prune_sample_kernel(const float* __restrict__ scores, int64_t n,
                                                            uint64_t seed, uint64_t step0, int n_draws,
                                                            uint32_t* __restrict__ keep) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float2 s = reinterpret_cast<const float2*>(scores)[i];
    const double d = (double)s.x - (double)s.y;
    const double g_min = -log(-log(0.5 / 16777216.0));
    const double u0_zero = exp(-exp(d - g_min)) - 1e-6;   // u0 below: the draw is 0
    const double u1_one = exp(-exp(-d - g_min)) - 1e-6;   // u1 below: the draw is 1
    uint32_t k = 0;
    for (int dr = 0; dr < n_draws && !k; ++dr) {
        const uint64_t step = step0 + (uint64_t)dr;
        uint32_t c0 = (uint32_t)i, c1 = (uint32_t)((uint64_t)i >> 32), c2 = (uint32_t)step,
                 c3 = (uint32_t)(step >> 32);
        philox4x32_10(c0, c1, c2, c3, (uint32_t)seed, (uint32_t)(seed >> 32));
        if (u01_from_bits(c0) < u0_zero) continue;
        if (u01_from_bits(c1) < u1_one) {
            k = 1u;
            break;
        }
        const double z0 = (double)s.x + gumbel_from_bits(c0);
        const double z1 = (double)s.y + gumbel_from_bits(c1);
        k = z0 > z1 ? 1u : 0u;
    }
    keep[i] = k;
}

// Stable compaction of per-Gaussian arrays: row i of every array goes to row
// pos[i] (exclusive scan of keep) when keep[i] != 0.  One launch covers up to
// CR_MAX arrays; each workgroup takes CR_ROWS rows of one array, stages their
// destinations in LDS, and moves the rows in units of `vec` floats (4, 2 or
// 1, as the width and the pointers' alignment allow).  Reads are coalesced
// over the workgroup's rows; writes are contiguous over runs of kept rows.
constexpr int CR_MAX = 32;
constexpr int CR_ROWS = RNT;
constexpr uint32_t CR_DROP = 0xffffffffu;

struct CompactSet {
    const float* in[CR_MAX];
    float* out[CR_MAX];
    uint32_t width[CR_MAX];
    uint32_t vec[CR_MAX];
    uint32_t block0[CR_MAX + 1];  // first workgroup of each array; block0[count] = grid size
    int count;
};

__global__ void __launch_bounds__(RNT) compact_rows_kernel(const uint32_t* __restrict__ keep,
                                                            const uint32_t* __restrict__ pos, int64_t n,
                                                            CompactSet cs) {
    __shared__ uint32_t s_dst[CR_ROWS];
    const uint32_t b = blockIdx.x;
    int a = 0;
    while (a + 1 < cs.count && cs.block0[a + 1] <= b) ++a;
    const int64_t r0 = (int64_t)(b - cs.block0[a]) * CR_ROWS;
    const int rows = (int)min((int64_t)CR_ROWS, n - r0);
    const int t = threadIdx.x;
    if (t < rows) s_dst[t] = keep[r0 + t] ? pos[r0 + t] : CR_DROP;
    __syncthreads();
    const uint32_t w = cs.width[a], vw = cs.vec[a], units = w / vw;
    const uint32_t total = (uint32_t)rows * units;
    const float* in = cs.in[a] + r0 * (int64_t)w;
    float* out = cs.out[a];
    for (uint32_t l = t; l < total; l += RNT) {
        const uint32_t r = l / units, c = l - r * units;
        const uint32_t d = s_dst[r];
        if (d == CR_DROP) continue;
        const int64_t src = (int64_t)l * vw, dst = (int64_t)d * w + (int64_t)c * vw;
        if (vw == 4) {
            *reinterpret_cast<float4*>(out + dst) = *reinterpret_cast<const float4*>(in + src);
        } else if (vw == 2) {
            *reinterpret_cast<float2*>(out + dst) = *reinterpret_cast<const float2*>(in + src);
        } else {
            out[dst] = in[src];
        }
    }
}

// Deterministic two-level sums in double.
__global__ void __launch_bounds__(RNT) partial_sum_kernel(const float* __restrict__ a, int64_t n,
                                                           double* __restrict__ partial) {
    __shared__ double sh[RNT / 64];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * RNT + threadIdx.x; i < n; i += (int64_t)gridDim.x * RNT) s += (double)a[i];
    s = block_sum_double(s, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// d (optional) receives sign(a - b) * inv_m, times *scale when scale is given
// (the upstream gradient of the loss, read on the device).
__global__ void __launch_bounds__(RNT) partial_abs_diff_kernel(const float* __restrict__ a,
                                                                const float* __restrict__ b, int64_t n,
                                                                float inv_m, const float* __restrict__ scale,
                                                                float* __restrict__ d,
                                                                double* __restrict__ partial) {
    __shared__ double sh[RNT / 64];
    if (scale) inv_m *= *scale;
    const bool write = d != nullptr;
    double s = 0.0;
    const int64_t stride = (int64_t)gridDim.x * RNT;
    int64_t head = 0;  // elements before this index go four at a time
    if ((((uintptr_t)a | (uintptr_t)b | (uintptr_t)d) & 15) == 0) {
        head = n & ~(int64_t)3;
        for (int64_t q = (int64_t)blockIdx.x * RNT + threadIdx.x; 4 * q < head; q += stride) {
            const float4 x = reinterpret_cast<const float4*>(a)[q], y = reinterpret_cast<const float4*>(b)[q];
            const float xs[4] = {x.x, x.y, x.z, x.w}, ys[4] = {y.x, y.y, y.z, y.w};
            float o[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const float e = xs[k] - ys[k];
                s += fabs((double)xs[k] - (double)ys[k]);
                o[k] = e > 0.f ? inv_m : (e < 0.f ? -inv_m : 0.f);
            }
            if (write) reinterpret_cast<float4*>(d)[q] = make_float4(o[0], o[1], o[2], o[3]);
        }
    }
    for (int64_t i = head + (int64_t)blockIdx.x * RNT + threadIdx.x; i < n; i += stride) {
        const float x = a[i] - b[i];
        s += fabs((double)a[i] - (double)b[i]);
        if (write) d[i] = x > 0.f ? inv_m : (x < 0.f ? -inv_m : 0.f);
    }
    s = block_sum_double(s, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void __launch_bounds__(RNT) finish_sum_kernel(const double* __restrict__ partial, int nb, double scale,
                                                          double* __restrict__ total, float* __restrict__ out_f,
                                                          int square) {
    __shared__ double sh[RNT / 64];
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += RNT) s += partial[i];
    s = block_sum_double(s, sh);
    if (threadIdx.x == 0) {
        *total = s;
        if (out_f) {
            const double m = s * scale;
            *out_f = (float)(square ? m * m : m);
        }
    }
}

__global__ void __launch_bounds__(RNT) mask_grad_kernel(const float* __restrict__ d_masks,
                                                         const float* __restrict__ y_soft, int64_t n, float tau,
                                                         float lambda_m, const float* __restrict__ lambda_scale,
                                                         const double* __restrict__ sum_m,
                                                         float* __restrict__ d_scores) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    // the weight of L_m in L (Eq. 8), optionally scaled by a device value (the
    // incoming gradient of L_m under autograd)
    if (lambda_scale) lambda_m *= *lambda_scale;
    // d L_m / d M_i = 2 mean(M) / n
    const float dlm = (float)(2.0 * (*sum_m) / ((double)n * (double)n));
    const float y = y_soft[i];
    const float g = (d_masks[i] + lambda_m * dlm) * y * (1.f - y) / tau;
    reinterpret_cast<float2*>(d_scores)[i] = make_float2(g, -g);
}

__global__ void __launch_bounds__(RNT) adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                                                    float* __restrict__ m, float* __restrict__ v, int64_t n, float lr,
                                                    float b1, float b2, float eps, float inv_c1, float inv_c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * inv_c1) / (sqrtf(vi * inv_c2) + eps);
}

// Adam over up to AM_MAX arrays in one launch.  Array j owns the blocks
// [block0[j], block0[j + 1]); each block updates AM_CHUNK consecutive
// elements.  The bias corrections use the step t = step + *step_off, read on
// the device, so a captured step advances with a device counter.
constexpr int AM_MAX = 16;
constexpr int AM_PER_THREAD = 16;
constexpr int64_t AM_CHUNK = (int64_t)RNT * AM_PER_THREAD;
struct AdamSet {
    float* p[AM_MAX];
    const float* g[AM_MAX];
    float* m[AM_MAX];
    float* v[AM_MAX];
    int64_t n[AM_MAX];
    float lr[AM_MAX];
    uint32_t vec[AM_MAX];  // 1: every pointer 16-byte aligned
    uint32_t block0[AM_MAX + 1];
    int count;
};

__device__ __forceinline__ void adam_one(float& p, float g, float& m, float& v, float lr, float b1, float b2,
                                         float eps, float inv_c1, float inv_c2) {
    m = b1 * m + (1.f - b1) * g;
    v = b2 * v + (1.f - b2) * g * g;
    p -= lr * (m * inv_c1) / (sqrtf(v * inv_c2) + eps);
}

__global__ void __launch_bounds__(RNT) adam_multi_kernel(AdamSet set, float b1, float b2, float eps, int64_t step,
                                                          const int64_t* __restrict__ step_off) {
    __shared__ float corr[2];
    int j = 0;
    while (j + 1 < set.count && blockIdx.x >= set.block0[j + 1]) ++j;
    if (threadIdx.x == 0) {
        const double t = (double)(step + (step_off ? *step_off : 0));
        corr[0] = (float)(1.0 / (1.0 - pow((double)b1, t)));
        corr[1] = (float)(1.0 / (1.0 - pow((double)b2, t)));
    }
    __syncthreads();
    const float inv_c1 = corr[0], inv_c2 = corr[1];
    const int64_t n = set.n[j];
    const float lr = set.lr[j];
    float* __restrict__ P = set.p[j];
    const float* __restrict__ G = set.g[j];
    float* __restrict__ Mo = set.m[j];
    float* __restrict__ Vo = set.v[j];
    const int64_t base = (int64_t)(blockIdx.x - set.block0[j]) * AM_CHUNK;
#pragma unroll
    for (int k = 0; k < AM_PER_THREAD / 4; ++k) {
        const int64_t i = base + 4 * ((int64_t)k * RNT + threadIdx.x);
        if (i >= n) break;
        if (set.vec[j] && i + 4 <= n) {
            float4 p = *reinterpret_cast<const float4*>(P + i);
            const float4 g = *reinterpret_cast<const float4*>(G + i);
            float4 m = *reinterpret_cast<const float4*>(Mo + i);
            float4 v = *reinterpret_cast<const float4*>(Vo + i);
            adam_one(p.x, g.x, m.x, v.x, lr, b1, b2, eps, inv_c1, inv_c2);
            adam_one(p.y, g.y, m.y, v.y, lr, b1, b2, eps, inv_c1, inv_c2);
            adam_one(p.z, g.z, m.z, v.z, lr, b1, b2, eps, inv_c1, inv_c2);
            adam_one(p.w, g.w, m.w, v.w, lr, b1, b2, eps, inv_c1, inv_c2);
            *reinterpret_cast<float4*>(P + i) = p;
            *reinterpret_cast<float4*>(Mo + i) = m;
            *reinterpret_cast<float4*>(Vo + i) = v;
        } else {
            const int64_t e = i + 4 < n ? i + 4 : n;
            for (int64_t q = i; q < e; ++q) {
                float p = P[q], m = Mo[q], v = Vo[q];
                adam_one(p, G[q], m, v, lr, b1, b2, eps, inv_c1, inv_c2);
                P[q] = p;
                Mo[q] = m;
                Vo[q] = v;
            }
        }
    }
}

__global__ void step_advance_kernel(int64_t* __restrict__ counter, int64_t delta) {
    if (threadIdx.x == 0) counter[0] += delta;
}

constexpr int REDUCE_BLOCKS = 1024;

}  // namespace

size_t reduce_scratch_bytes(int64_t) { return (REDUCE_BLOCKS + 8) * sizeof(double); }

void launch_sample_masks(hipStream_t stream, const float* scores, int64_t n, float tau, uint64_t seed, uint64_t step,
                         const uint64_t* step_off, float* m_hard, float* y_soft) {
    if (n == 0) return;
    hipLaunchKernelGGL(sample_masks_kernel, dim3((unsigned)((n + RNT - 1) / RNT)), dim3(RNT), 0, stream, scores, n,
                       tau, seed, step, step_off, m_hard, y_soft);
}

void launch_threshold_masks(hipStream_t stream, const float* scores, int64_t n, double threshold, float* m_hard,
                            float* y_soft) {
    if (n == 0) return;
    hipLaunchKernelGGL(threshold_masks_kernel, dim3((unsigned)((n + RNT - 1) / RNT)), dim3(RNT), 0, stream, scores,
                       n, threshold, m_hard, y_soft);
}

void launch_prune_sample(hipStream_t stream, const float* scores, int64_t n, uint64_t seed, uint64_t step0,
                         int n_draws, uint32_t* keep) {
    if (n == 0) return;
    hipLaunchKernelGGL(prune_sample_kernel, dim3((unsigned)((n + RNT - 1) / RNT)), dim3(RNT), 0, stream, scores, n,
                       seed, step0, n_draws, keep);
}

void launch_compact_rows(hipStream_t stream, const uint32_t* keep, const uint32_t* pos, int64_t n, int n_arrays,
                         const float* const* in, float* const* out, const int* widths) {
    if (n == 0) return;
    const uint32_t per = (uint32_t)((n + CR_ROWS - 1) / CR_ROWS);
    for (int a0 = 0; a0 < n_arrays; a0 += CR_MAX) {
        CompactSet cs{};
        cs.count = min(CR_MAX, n_arrays - a0);
        for (int j = 0; j < cs.count; ++j) {
            const int a = a0 + j;
            const uint32_t w = (uint32_t)widths[a];
            const uintptr_t al = (uintptr_t)in[a] | (uintptr_t)out[a];
            cs.in[j] = in[a];
            cs.out[j] = out[a];
            cs.width[j] = w;
            cs.vec[j] = (w % 4 == 0 && al % 16 == 0) ? 4u : (w % 2 == 0 && al % 8 == 0) ? 2u : 1u;
            cs.block0[j] = (uint32_t)j * per;
        }
        cs.block0[cs.count] = (uint32_t)cs.count * per;
        hipLaunchKernelGGL(compact_rows_kernel, dim3(cs.block0[cs.count]), dim3(RNT), 0, stream, keep, pos, n, cs);
    }
}

// (mean M)^2 into loss_m (optional); the double sum of M stays in the
// scratch for the gradient.
static const double* mask_sum(hipStream_t stream, const float* m_hard, int64_t n, float* loss_m, void* scratch) {
    double* partial = reinterpret_cast<double*>(scratch);
    double* total = partial + REDUCE_BLOCKS;
    const int nb = (int)std::min<int64_t>(REDUCE_BLOCKS, (n + RNT - 1) / RNT);
    hipLaunchKernelGGL(partial_sum_kernel, dim3(nb), dim3(RNT), 0, stream, m_hard, n, partial);
    hipLaunchKernelGGL(finish_sum_kernel, dim3(1), dim3(RNT), 0, stream, (const double*)partial, nb, 1.0 / (double)n,
                       total, loss_m, 1);
    return total;
}

void launch_mask_loss(hipStream_t stream, const float* m_hard, int64_t n, float* loss_m, void* scratch) {
    if (n == 0) {
        launch_fill_f32(stream, loss_m, 1, 0.f);
        return;
    }
    (void)mask_sum(stream, m_hard, n, loss_m, scratch);
}

void launch_mask_grad(hipStream_t stream, const float* d_masks, const float* m_hard, const float* y_soft, int64_t n,
                      float tau, float lambda_m, const float* lambda_scale, float* d_scores, float* loss_m,
                      void* scratch) {
    if (n == 0) return;
    const double* total = mask_sum(stream, m_hard, n, loss_m, scratch);
    hipLaunchKernelGGL(mask_grad_kernel, dim3((unsigned)((n + RNT - 1) / RNT)), dim3(RNT), 0, stream, d_masks, y_soft,
                       n, tau, lambda_m, lambda_scale, total, d_scores);
}

void launch_l1_loss_grad(hipStream_t stream, const float* images, const float* targets, int64_t m, float* d_images,
                         const float* grad_scale, float* loss, void* scratch) {
    if (m == 0) return;
    double* partial = reinterpret_cast<double*>(scratch);
    double* total = partial + REDUCE_BLOCKS;
    const int nb = (int)std::min<int64_t>(REDUCE_BLOCKS, (m + RNT - 1) / RNT);
    hipLaunchKernelGGL(partial_abs_diff_kernel, dim3(nb), dim3(RNT), 0, stream, images, targets, m,
                       (float)(1.0 / (double)m), grad_scale, d_images, partial);
    if (loss)
        hipLaunchKernelGGL(finish_sum_kernel, dim3(1), dim3(RNT), 0, stream, (const double*)partial, nb,
                           1.0 / (double)m, total, loss, 0);
}

int adam_multi_max() { return AM_MAX; }

void launch_adam_multi(hipStream_t stream, const AdamArray* arrays, int n_arrays, float b1, float b2, float eps,
                       int64_t step, const int64_t* step_off) {
    for (int a0 = 0; a0 < n_arrays; a0 += AM_MAX) {
        AdamSet set{};
        set.count = 0;
        uint32_t blocks = 0;
        for (int j = 0; j < AM_MAX && a0 + j < n_arrays; ++j) {
            const AdamArray& x = arrays[a0 + j];
            if (x.n <= 0) continue;
            const int k = set.count++;
            set.p[k] = x.params;
            set.g[k] = x.grads;
            set.m[k] = x.m;
            set.v[k] = x.v;
            set.n[k] = x.n;
            set.lr[k] = x.lr;
            const uintptr_t al = (uintptr_t)x.params | (uintptr_t)x.grads | (uintptr_t)x.m | (uintptr_t)x.v;
            set.vec[k] = (al & 15) == 0 ? 1u : 0u;
            set.block0[k] = blocks;
            blocks += (uint32_t)((x.n + AM_CHUNK - 1) / AM_CHUNK);
        }
        if (set.count == 0) continue;
        set.block0[set.count] = blocks;
        hipLaunchKernelGGL(adam_multi_kernel, dim3(blocks), dim3(RNT), 0, stream, set, b1, b2, eps, step, step_off);
    }
}

void launch_step_advance(hipStream_t stream, int64_t* counter, int64_t delta) {
    hipLaunchKernelGGL(step_advance_kernel, dim3(1), dim3(64), 0, stream, counter, delta);
}

void launch_adam(hipStream_t stream, float* params, const float* grads, float* m, float* v, int64_t n, float lr,
                 float b1, float b2, float eps, int64_t step) {
    if (n == 0) return;
    const double c1 = 1.0 - pow((double)b1, (double)step), c2 = 1.0 - pow((double)b2, (double)step);
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + RNT - 1) / RNT)), dim3(RNT), 0, stream, params, grads, m, v,
                       n, lr, b1, b2, eps, (float)(1.0 / c1), (float)(1.0 / c2));
}

}  // namespace mgs
