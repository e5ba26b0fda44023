// EWA projection of 3D Gaussians and its backward pass (gfx950).
//
// Forward (Sec. 3.1): scale/quaternion -> 3D covariance, view transform,
// perspective Jacobian -> 2D covariance (+ dilation) -> conic, radius, tile
// footprint, and the view-dependent SH colour.  Masks are not applied here;
// they only travel in the record to the compositing kernels (Sec. 3.2-3.3).
//
// One thread per Gaussian loops over all views, so the 3D covariance and
// the SH coefficients (up to 192 B) are read from HBM once per Gaussian
// rather than once per view.
//
// The covariance chain (3D covariance, Jacobian, 2D covariance, its inverse,
// and their derivatives) runs in double precision: needle-shaped Gaussians
// (scale ratios of 1e4 and more) lose their thin direction in FP32 and can
// produce a negative 2D determinant.  Vector FP64 runs at the lane rate of
// non-packed FP32 on this chip, and these kernels are bound by HBM traffic.
// Colours (SH) are FP32.
#include "common.hpp"
#include "kernels.hpp"

namespace mgs {
namespace {

// Real spherical harmonics (no Condon-Shortley phase) in Cartesian form.
constexpr float SH0 = 0.28209479177387814f;   // 1 / (2 sqrt(pi))
constexpr float SH1 = 0.48860251190291992f;   // sqrt(3 / (4 pi))
constexpr float SH2a = 1.0925484305920792f;   // sqrt(15 / pi) / 2
constexpr float SH2b = 0.31539156525252005f;  // sqrt(5 / pi) / 4
constexpr float SH2c = 0.54627421529603959f;  // sqrt(15 / pi) / 4
constexpr float SH3a = 0.59004358992664352f;  // sqrt(35 / (2 pi)) / 4
constexpr float SH3b = 2.8906114426405538f;   // sqrt(105 / pi) / 2
constexpr float SH3c = 0.45704579946446572f;  // sqrt(21 / (2 pi)) / 4
constexpr float SH3d = 0.37317633259011540f;  // sqrt(7 / pi) / 4
constexpr float SH3e = 1.4453057213202769f;   // sqrt(105 / pi) / 4

template <int DEG>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float* Y) {
    Y[0] = SH0;
    if (DEG >= 1) {
        Y[1] = SH1 * y;
        Y[2] = SH1 * z;
        Y[3] = SH1 * x;
    }
    if (DEG >= 2) {
        Y[4] = SH2a * x * y;
        Y[5] = SH2a * y * z;
        Y[6] = SH2b * (3.f * z * z - 1.f);
        Y[7] = SH2a * x * z;
        Y[8] = SH2c * (x * x - y * y);
    }
    if (DEG >= 3) {
        Y[9] = SH3a * y * (3.f * x * x - y * y);
        Y[10] = SH3b * x * y * z;
        Y[11] = SH3c * y * (5.f * z * z - 1.f);
        Y[12] = SH3d * z * (5.f * z * z - 3.f);
        Y[13] = SH3c * x * (5.f * z * z - 1.f);
        Y[14] = SH3e * z * (x * x - y * y);
        Y[15] = SH3a * x * (x * x - 3.f * y * y);
    }
}

// Partial derivatives of the polynomials above in (x, y, z).
template <int DEG>
__device__ __forceinline__ void sh_basis_grad(float x, float y, float z, float (*D)[3]) {
    D[0][0] = D[0][1] = D[0][2] = 0.f;
    if (DEG >= 1) {
        D[1][0] = 0.f;  D[1][1] = SH1;  D[1][2] = 0.f;
        D[2][0] = 0.f;  D[2][1] = 0.f;  D[2][2] = SH1;
        D[3][0] = SH1;  D[3][1] = 0.f;  D[3][2] = 0.f;
    }
    if (DEG >= 2) {
        D[4][0] = SH2a * y;        D[4][1] = SH2a * x;         D[4][2] = 0.f;
        D[5][0] = 0.f;             D[5][1] = SH2a * z;         D[5][2] = SH2a * y;
        D[6][0] = 0.f;             D[6][1] = 0.f;              D[6][2] = SH2b * 6.f * z;
        D[7][0] = SH2a * z;        D[7][1] = 0.f;              D[7][2] = SH2a * x;
        D[8][0] = SH2c * 2.f * x;  D[8][1] = -SH2c * 2.f * y;  D[8][2] = 0.f;
    }
    if (DEG >= 3) {
        D[9][0] = SH3a * 6.f * x * y;
        D[9][1] = SH3a * 3.f * (x * x - y * y);
        D[9][2] = 0.f;
        D[10][0] = SH3b * y * z;
        D[10][1] = SH3b * x * z;
        D[10][2] = SH3b * x * y;
        D[11][0] = 0.f;
        D[11][1] = SH3c * (5.f * z * z - 1.f);
        D[11][2] = SH3c * 10.f * y * z;
        D[12][0] = 0.f;
        D[12][1] = 0.f;
        D[12][2] = SH3d * (15.f * z * z - 3.f);
        D[13][0] = SH3c * (5.f * z * z - 1.f);
        D[13][1] = 0.f;
        D[13][2] = SH3c * 10.f * x * z;
        D[14][0] = SH3e * 2.f * x * z;
        D[14][1] = -SH3e * 2.f * y * z;
        D[14][2] = SH3e * (x * x - y * y);
        D[15][0] = SH3a * 3.f * (x * x - y * y);
        D[15][1] = -SH3a * 6.f * x * y;
        D[15][2] = 0.f;
    }
}

template <int DEG>
__device__ __forceinline__ void load_sh(const float* __restrict__ sh, int64_t g, float* c) {
    constexpr int K3 = 3 * (DEG + 1) * (DEG + 1);
    const float* p = sh + g * K3;
    if constexpr (K3 % 4 == 0) {
        const float4* p4 = reinterpret_cast<const float4*>(p);
#pragma unroll
        for (int i = 0; i < K3 / 4; ++i) {
            const float4 q = p4[i];
            c[4 * i] = q.x; c[4 * i + 1] = q.y; c[4 * i + 2] = q.z; c[4 * i + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < K3; ++i) c[i] = p[i];
    }
}

// Scale, rotation and 3D covariance of one Gaussian, in double.
struct Cov3 {
    double s[3];
    double q[4];     // normalised (w, x, y, z)
    double qinv;     // 1 / |q|
    double R[9];     // rotation, row-major
    double S[6];     // covariance entries 00, 01, 02, 11, 12, 22
};

__device__ __forceinline__ Cov3 cov3_of(float l0, float l1, float l2, float4 q4) {
    Cov3 c;
    c.s[0] = exp((double)l0);
    c.s[1] = exp((double)l1);
    c.s[2] = exp((double)l2);
    const double qw = q4.x, qx = q4.y, qy = q4.z, qz = q4.w;
    c.qinv = 1.0 / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    const double w = qw * c.qinv, x = qx * c.qinv, y = qy * c.qinv, z = qz * c.qinv;
    c.q[0] = w; c.q[1] = x; c.q[2] = y; c.q[3] = z;
    c.R[0] = 1.0 - 2.0 * (y * y + z * z); c.R[1] = 2.0 * (x * y - w * z);       c.R[2] = 2.0 * (x * z + w * y);
    c.R[3] = 2.0 * (x * y + w * z);       c.R[4] = 1.0 - 2.0 * (x * x + z * z); c.R[5] = 2.0 * (y * z - w * x);
    c.R[6] = 2.0 * (x * z - w * y);       c.R[7] = 2.0 * (y * z + w * x);       c.R[8] = 1.0 - 2.0 * (x * x + y * y);
    double M[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) M[3 * i + k] = c.R[3 * i + k] * c.s[k];
    c.S[0] = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
    c.S[1] = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
    c.S[2] = M[0] * M[6] + M[1] * M[7] + M[2] * M[8];
    c.S[3] = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
    c.S[4] = M[3] * M[6] + M[4] * M[7] + M[5] * M[8];
    c.S[5] = M[6] * M[6] + M[7] * M[7] + M[8] * M[8];
    return c;
}

__device__ __forceinline__ Cov3 cov3(const float* __restrict__ log_scales, const float* __restrict__ quats,
                                     int64_t g) {
    return cov3_of(log_scales[3 * g], log_scales[3 * g + 1], log_scales[3 * g + 2],
                   reinterpret_cast<const float4*>(quats)[g]);
}

struct ViewGeom {
    bool valid;
    float depth;          // float32 of the double view-space z (sort key, cull test)
    double tx, ty, tz;    // view-space centre
    float u, v;
    double sx, sy;        // lateral ratios after clamping
    bool clx, cly;
    double T0[3], T1[3];  // J W
    double a, b, c;       // 2D covariance incl. dilation
    double detv;          // its determinant
    double ca;            // conic entry a = c / det
    double beta, gamma;   // conic stored as (ca, cb / ca, cc - cb^2 / ca) = (ca, -b / c, 1 / c)
    float radius;
};

// Per-view geometry of one Gaussian.  FULL = false stops after the 2D
// covariance and its determinant (the conic, the radius and their finiteness
// test are left unset): for a record the forward already found valid, whose
// tests this double computation would repeat bit for bit.
template <bool FULL = true>
__device__ __forceinline__ ViewGeom view_geom(const DevView& cam, const DevSettings& st, float px, float py, float pz,
                                              const double* Sig) {
    ViewGeom o;
    // products of two floats are exact in double, so the association
    // ((W0 x + W1 y) + W2 z) + t fixes the depth key bit for bit
    const double xd = px, yd = py, zd = pz;
    o.tx = (((double)cam.W[0] * xd + (double)cam.W[1] * yd) + (double)cam.W[2] * zd) + (double)cam.t[0];
    o.ty = (((double)cam.W[3] * xd + (double)cam.W[4] * yd) + (double)cam.W[5] * zd) + (double)cam.t[1];
    o.tz = (((double)cam.W[6] * xd + (double)cam.W[7] * yd) + (double)cam.W[8] * zd) + (double)cam.t[2];
    o.depth = (float)o.tz;
    o.valid = o.depth > st.near_plane;
    if (!o.valid) return o;
    const double fx = cam.fx, fy = cam.fy;
    const double iz = 1.0 / o.tz;
    o.u = (float)(fx * o.tx * iz + (double)cam.cx);
    o.v = (float)(fy * o.ty * iz + (double)cam.cy);
    const double limx = cam.limx, limy = cam.limy;
    const double rx = o.tx * iz, ry = o.ty * iz;
    o.clx = rx < -limx || rx > limx;
    o.cly = ry < -limy || ry > limy;
    o.sx = fmin(fmax(rx, -limx), limx);
    o.sy = fmin(fmax(ry, -limy), limy);
    const double J00 = fx * iz, J02 = -fx * o.sx * iz;
    const double J11 = fy * iz, J12 = -fy * o.sy * iz;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        o.T0[j] = J00 * (double)cam.W[j] + J02 * (double)cam.W[6 + j];
        o.T1[j] = J11 * (double)cam.W[3 + j] + J12 * (double)cam.W[6 + j];
    }
    const double S00 = Sig[0], S01 = Sig[1], S02 = Sig[2], S11 = Sig[3], S12 = Sig[4], S22 = Sig[5];
    const double U00 = o.T0[0] * S00 + o.T0[1] * S01 + o.T0[2] * S02;
    const double U01 = o.T0[0] * S01 + o.T0[1] * S11 + o.T0[2] * S12;
    const double U02 = o.T0[0] * S02 + o.T0[1] * S12 + o.T0[2] * S22;
    const double U10 = o.T1[0] * S00 + o.T1[1] * S01 + o.T1[2] * S02;
    const double U11 = o.T1[0] * S01 + o.T1[1] * S11 + o.T1[2] * S12;
    const double U12 = o.T1[0] * S02 + o.T1[1] * S12 + o.T1[2] * S22;
    const double dil = st.dilation;
    o.a = U00 * o.T0[0] + U01 * o.T0[1] + U02 * o.T0[2] + dil;
    o.b = U00 * o.T1[0] + U01 * o.T1[1] + U02 * o.T1[2];
    o.c = U10 * o.T1[0] + U11 * o.T1[1] + U12 * o.T1[2] + dil;
    const double det = o.a * o.c - o.b * o.b;
    if (!(det > 0.0)) { o.valid = false; return o; }
    o.detv = det;
    if (!FULL) return o;
    o.ca = o.c / det;
    o.beta = -o.b / o.c;
    o.gamma = 1.0 / o.c;
    const double mid = 0.5 * (o.a + o.c);
    const double disc = fmax((double)st.lambda_floor, mid * mid - det);
    o.radius = (float)ceil(3.0 * sqrt(mid + sqrt(disc)));
    if (!(isfinite(o.u) && isfinite(o.v) && isfinite((float)o.ca) && isfinite((float)o.beta) &&
          isfinite((float)o.gamma) && isfinite(o.radius) && o.radius > 0.f))
        o.valid = false;
    return o;
}

template <int DEG>
__global__ void __launch_bounds__(256) project_fwd_kernel(
    const float* __restrict__ means, const float* __restrict__ log_scales, const float* __restrict__ quats,
    const float* __restrict__ opacity_logits, const float* __restrict__ sh, const float* __restrict__ masks,
    int64_t n, ViewSet views, DevSettings st, float4* __restrict__ rec, float* __restrict__ depth_out,
    float* __restrict__ radius_out, uint32_t* __restrict__ tiles_out, uint32_t* __restrict__ flags,
    uint32_t* __restrict__ rkeys, uint32_t* __restrict__ rvals) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const float px = means[3 * g], py = means[3 * g + 1], pz = means[3 * g + 2];
    const Cov3 cv = cov3(log_scales, quats, g);
    const float opac_raw = 1.f / (1.f + __expf(-opacity_logits[g]));
    // mask x opacity (the ablation's alternative): the record's opacity is
    // M * sigmoid(logit) and its mask 1; masked rasterization keeps them apart
    const float opac = st.mask_opacity ? masks[g] * opac_raw : opac_raw;
    const float mval = st.mask_opacity ? 1.f : masks[g];
    float coef[3 * K];
    load_sh<DEG>(sh, g, coef);
    bool bad = false;
    for (int vi = 0; vi < views.n_views; ++vi) {
        const DevView& cam = views.v[vi];
        const int64_t r = (int64_t)vi * n + g;
        const ViewGeom o = view_geom(cam, st, px, py, pz, cv.S);
        if (!o.valid) {
            // culled; flagged as non-finite unless simply behind the near plane
            if (o.depth > st.near_plane) bad = true;
            rec[3 * r] = make_float4(0.f, 0.f, 0.f, 0.f);
            rec[3 * r + 1] = make_float4(0.f, 0.f, 0.f, 0.f);
            rec[3 * r + 2] = make_float4(0.f, 0.f, 0.f, 0.f);
            depth_out[r] = o.depth;
            if (radius_out) radius_out[r] = 0.f;
            tiles_out[r] = 0;
            if (rkeys) {
                rkeys[r] = 0xffffffffu;
                rvals[r] = (uint32_t)r;
            }
            continue;
        }
        // colour in the viewing direction
        float dx = px - cam.campos[0], dy = py - cam.campos[1], dz = pz - cam.campos[2];
        const float dinv = rsqrtf(dx * dx + dy * dy + dz * dz);
        dx *= dinv; dy *= dinv; dz *= dinv;
        float Y[K];
        sh_basis<DEG>(dx, dy, dz, Y);
        float col[3];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            float acc = 0.5f;
#pragma unroll
            for (int k = 0; k < K; ++k) acc += coef[3 * k + ch] * Y[k];
            col[ch] = fmaxf(acc, 0.f);
        }
        // square footprint in tiles, in double so the bounds are exact
        uint32_t count;
        if (st.full_rect) {
            count = (uint32_t)(cam.grid_w * cam.grid_h);
        } else {
            const double ud = o.u, vd = o.v, rd = o.radius;
            // tile sizes are powers of two: ldexp by -log2 equals the division
            const int kw = __builtin_ctz((unsigned)st.tile_w), kh = __builtin_ctz((unsigned)st.tile_h);
            double x0 = floor(ldexp(ud - rd, -kw)), x1 = floor(ldexp(ud + rd, -kw));
            double y0 = floor(ldexp(vd - rd, -kh)), y1 = floor(ldexp(vd + rd, -kh));
            x0 = fmax(x0, 0.0); y0 = fmax(y0, 0.0);
            x1 = fmin(x1, (double)(cam.grid_w - 1)); y1 = fmin(y1, (double)(cam.grid_h - 1));
            count = (x0 <= x1 && y0 <= y1) ? (uint32_t)((x1 - x0 + 1.0) * (y1 - y0 + 1.0)) : 0u;
        }
        rec[3 * r] = make_float4(o.u, o.v, (float)o.ca, (float)o.beta);
        rec[3 * r + 1] = make_float4((float)o.gamma, opac, mval, o.radius);
        rec[3 * r + 2] = make_float4(col[0], col[1], col[2], __uint_as_float(count));
        depth_out[r] = o.depth;
        if (radius_out) radius_out[r] = o.radius;  // (also in the record, B.w)
        tiles_out[r] = count;
        // keys of the depth order of the records (per view): the depth bits,
        // all ones for a record listed nowhere (sorted last in its view)
        if (rkeys) {
            rkeys[r] = count ? __float_as_uint(o.depth) : 0xffffffffu;
            rvals[r] = (uint32_t)r;
        }
    }
    if (bad) atomicOr(flags, FLAG_NONFINITE);
}

// out[r] = field f (0..11) of record r: the radius export reads B.w (f = 7)
__global__ void __launch_bounds__(256) record_field_kernel(const float* __restrict__ rec, int64_t R, int f,
                                                            float* __restrict__ out) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < R) out[r] = rec[12 * r + f];
}

// AccT: type of the per-record 2D gradients (float from the stage entry
// point, double from the whole path, which accumulates them with FP64
// atomics); dm_acc (optional) holds FP64 mask gradients to round into d_masks.
// clear (optional, the same array as d_rec): each row read is set back to
// zero, so the accumulator is clean for the next backward without a fill
// (only records listed in some tile can have received gradients, and every
// such row is read here).  tiles (optional): the forward's per-record tile
// counts; rows of records without tiles are neither read nor cleared.
// TILES: tiles is given (a listed record then passed the forward's validity
// tests on the same double values, which are not repeated).
template <int DEG, typename AccT, bool ACC, bool TILES>
__global__ void __launch_bounds__(256) project_bwd_kernel(
    const float* __restrict__ means, const float* __restrict__ log_scales, const float* __restrict__ quats,
    const float* __restrict__ opacity_logits, const float* __restrict__ sh, const float* __restrict__ masks,
    int64_t n, ViewSet views, DevSettings st, const AccT* d_rec, const double* __restrict__ dm_acc, AccT* clear,
    float* __restrict__ d_means,
    float* __restrict__ d_log_scales, float* __restrict__ d_quats, float* __restrict__ d_opacity_logits,
    float* __restrict__ d_sh, float* __restrict__ d_masks, float* __restrict__ d_rec_out,
    const uint32_t* __restrict__ tiles) {
    constexpr int K = (DEG + 1) * (DEG + 1);
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    // ACC: parameter gradients are added to what the outputs hold (a
    // template parameter: the overwriting kernel keeps its vector stores)
    constexpr bool accumulate = ACC;
    const float px = means[3 * g], py = means[3 * g + 1], pz = means[3 * g + 2];
    const float opac = 1.f / (1.f + __expf(-opacity_logits[g]));
    // Two passes over the views, so that the double-precision covariance
    // chain and the SH colour (coefficients and their gradients) are never
    // live together: one pass holding both needs more than 256 registers,
    // which leaves one wave per SIMD.  The first pass reads each valid
    // view's whole gradient row once (and clears it when asked to), keeping
    // the colour gradients in LDS (3 floats per view and thread) for the
    // second.
    extern __shared__ float s_dcol[];  // [n_views][3][blockDim.x]
    const int tid = threadIdx.x, nth = blockDim.x;
    uint32_t valid = 0;
    double gp[3] = {0.0, 0.0, 0.0};
    double gop = 0.0;
    {
        // the loop needs the 3D covariance only; rotation and scales are
        // formed again after it
        double Sig[6];
        {
            const Cov3 c0 = cov3(log_scales, quats, g);
#pragma unroll
            for (int i = 0; i < 6; ++i) Sig[i] = c0.S[i];
        }
        double gS[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // dL/dSigma3 (symmetric full-matrix gradient)
        for (int vi = 0; vi < views.n_views; ++vi) {
            const DevView& cam = views.v[vi];
            const int64_t r = (int64_t)vi * n + g;
            // a record without tiles (every invalid one among them) was listed
            // nowhere: its row was never written and is zero (tiles: the
            // forward's per-record counts); its geometry is not formed
            const bool listed = !TILES || tiles[r] != 0u;
            // with the tile counts, a listed record passed the forward's
            // validity tests on the same double values: only the geometry
            // the gradients use is formed again
            ViewGeom o;
            if (listed) o = view_geom<!TILES>(cam, st, px, py, pz, Sig);
            if (!listed || !o.valid) {
                if (d_rec_out) {
#pragma unroll
                    for (int q = 0; q < DREC; ++q) d_rec_out[r * DREC + q] = 0.f;
                }
                continue;
            }
            valid |= 1u << vi;
            const AccT* dr = d_rec + r * DREC;
            if (d_rec_out) {
#pragma unroll
                for (int q = 0; q < DREC; ++q) d_rec_out[r * DREC + q] = (float)dr[q];
            }
            const double du = dr[0], dv = dr[1], dca = dr[2], dcb = dr[3], dcc = dr[4];
            gop += (double)dr[5];
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) s_dcol[(vi * 3 + ch) * nth + tid] = (float)dr[6 + ch];
            if (clear) {
#pragma unroll
                for (int q = 0; q < DREC; ++q) clear[r * DREC + q] = (AccT)0;
            }
            // stored conic (a, beta, gamma) = (c / det, -b / c, 1 / c) of the 2D
            // covariance [[a, b], [b, c]] -> H = dL/dcov2D (symmetric, H01 is half
            // the derivative w.r.t. the shared off-diagonal entry).  The per-pixel
            // sums arrive in this basis because it keeps the thin direction of a
            // needle apart from the long one in FP32.
            const double s2 = o.c * o.c, idet2 = 1.0 / (o.detv * o.detv);
            const double H00 = -dca * s2 * idet2;
            const double H01 = 0.5 * (2.0 * dca * o.b * o.c * idet2 - dcb / o.c);
            const double H11 = (-dca * o.b * o.b * idet2 + dcb * o.b / s2) - dcc / s2;
            // dSigma3 += T^T H T ; dT = 2 H T Sigma3
            double HT0[3], HT1[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                HT0[j] = H00 * o.T0[j] + H01 * o.T1[j];
                HT1[j] = H01 * o.T0[j] + H11 * o.T1[j];
            }
            gS[0] += o.T0[0] * HT0[0] + o.T1[0] * HT1[0];
            gS[1] += o.T0[0] * HT0[1] + o.T1[0] * HT1[1];
            gS[2] += o.T0[0] * HT0[2] + o.T1[0] * HT1[2];
            gS[3] += o.T0[1] * HT0[1] + o.T1[1] * HT1[1];
            gS[4] += o.T0[1] * HT0[2] + o.T1[1] * HT1[2];
            gS[5] += o.T0[2] * HT0[2] + o.T1[2] * HT1[2];
            const double* S = Sig;
            double dT0[3], dT1[3];
            dT0[0] = 2.0 * (HT0[0] * S[0] + HT0[1] * S[1] + HT0[2] * S[2]);
            dT0[1] = 2.0 * (HT0[0] * S[1] + HT0[1] * S[3] + HT0[2] * S[4]);
            dT0[2] = 2.0 * (HT0[0] * S[2] + HT0[1] * S[4] + HT0[2] * S[5]);
            dT1[0] = 2.0 * (HT1[0] * S[0] + HT1[1] * S[1] + HT1[2] * S[2]);
            dT1[1] = 2.0 * (HT1[0] * S[1] + HT1[1] * S[3] + HT1[2] * S[4]);
            dT1[2] = 2.0 * (HT1[0] * S[2] + HT1[1] * S[4] + HT1[2] * S[5]);
            // T = J W  ->  dJ = dT W^T (only J00, J02, J11, J12 are variables)
            const double W0 = cam.W[0], W1 = cam.W[1], W2 = cam.W[2], W3 = cam.W[3], W4 = cam.W[4], W5 = cam.W[5];
            const double W6 = cam.W[6], W7 = cam.W[7], W8 = cam.W[8];
            const double dJ00 = dT0[0] * W0 + dT0[1] * W1 + dT0[2] * W2;
            const double dJ02 = dT0[0] * W6 + dT0[1] * W7 + dT0[2] * W8;
            const double dJ11 = dT1[0] * W3 + dT1[1] * W4 + dT1[2] * W5;
            const double dJ12 = dT1[0] * W6 + dT1[1] * W7 + dT1[2] * W8;
            // view-space centre
            const double fx = cam.fx, fy = cam.fy;
            const double iz = 1.0 / o.tz, iz2 = iz * iz;
            double dtx = du * fx * iz;
            double dty = dv * fy * iz;
            double dtz = -(du * fx * o.tx + dv * fy * o.ty) * iz2;
            dtz += -(dJ00 * fx + dJ11 * fy) * iz2;
            if (!o.clx) {
                dtx += -dJ02 * fx * iz2;
                dtz += dJ02 * 2.0 * fx * o.tx * iz2 * iz;
            } else {
                dtz += dJ02 * fx * o.sx * iz2;
            }
            if (!o.cly) {
                dty += -dJ12 * fy * iz2;
                dtz += dJ12 * 2.0 * fy * o.ty * iz2 * iz;
            } else {
                dtz += dJ12 * fy * o.sy * iz2;
            }
            // t = W p + t  ->  dp = W^T dt
            gp[0] += W0 * dtx + W3 * dty + W6 * dtz;
            gp[1] += W1 * dtx + W4 * dty + W7 * dtz;
            gp[2] += W2 * dtx + W5 * dty + W8 * dtz;
        }
        // the inputs pass through an empty asm statement, which hides from
        // the compiler that they equal the values loaded before the loop, so
        // it forms rotation and scales anew instead of keeping them live
        // (in registers) across the loop
        float l0 = log_scales[3 * g], l1 = log_scales[3 * g + 1], l2 = log_scales[3 * g + 2];
        float4 q4 = reinterpret_cast<const float4*>(quats)[g];
        asm volatile("" : "+v"(l0), "+v"(l1), "+v"(l2), "+v"(q4.x), "+v"(q4.y), "+v"(q4.z), "+v"(q4.w));
        const Cov3 cv = cov3_of(l0, l1, l2, q4);
        // Sigma3 = R diag(s^2) R^T with G = dL/dSigma3 (symmetric)
        const double G[9] = {gS[0], gS[1], gS[2], gS[1], gS[3], gS[4], gS[2], gS[4], gS[5]};
        const double* R = cv.R;
        double GR[9];  // G R
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int k = 0; k < 3; ++k) GR[3 * i + k] = G[3 * i] * R[k] + G[3 * i + 1] * R[3 + k] + G[3 * i + 2] * R[6 + k];
        double dR[9];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int k = 0; k < 3; ++k) dR[3 * i + k] = 2.0 * GR[3 * i + k] * cv.s[k] * cv.s[k];
        double dls[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double rgr = R[k] * GR[k] + R[3 + k] * GR[3 + k] + R[6 + k] * GR[6 + k];  // (R^T G R)_kk
            dls[k] = 2.0 * cv.s[k] * cv.s[k] * rgr;
        }
        // rotation matrix -> normalised quaternion -> raw quaternion
        const double qw = cv.q[0], qx = cv.q[1], qy = cv.q[2], qz = cv.q[3];
        const double gw = 2.0 * (-qz * dR[1] + qy * dR[2] + qz * dR[3] - qx * dR[5] - qy * dR[6] + qx * dR[7]);
        const double gx = 2.0 * (qy * dR[1] + qz * dR[2] + qy * dR[3] - 2.0 * qx * dR[4] - qw * dR[5] + qz * dR[6] +
                                 qw * dR[7] - 2.0 * qx * dR[8]);
        const double gy = 2.0 * (-2.0 * qy * dR[0] + qx * dR[1] + qw * dR[2] + qx * dR[3] + qz * dR[5] - qw * dR[6] +
                                 qz * dR[7] - 2.0 * qy * dR[8]);
        const double gz = 2.0 * (-2.0 * qz * dR[0] - qw * dR[1] + qx * dR[2] + qw * dR[3] - 2.0 * qz * dR[4] +
                                 qy * dR[5] + qx * dR[6] + qy * dR[7]);
        const double dotq = qw * gw + qx * gx + qy * gy + qz * gz;
        if (d_quats) {
            float4 dq = make_float4((float)((gw - qw * dotq) * cv.qinv), (float)((gx - qx * dotq) * cv.qinv),
                                    (float)((gy - qy * dotq) * cv.qinv), (float)((gz - qz * dotq) * cv.qinv));
            if constexpr (ACC) {
                const float4 o = reinterpret_cast<const float4*>(d_quats)[g];
                dq.x += o.x; dq.y += o.y; dq.z += o.z; dq.w += o.w;
            }
            reinterpret_cast<float4*>(d_quats)[g] = dq;
        }
        if (d_log_scales) {
#pragma unroll
            for (int k = 0; k < 3; ++k)
                d_log_scales[3 * g + k] = accumulate ? d_log_scales[3 * g + k] + (float)dls[k] : (float)dls[k];
        }
    }
    {
        float coef[3 * K];
        load_sh<DEG>(sh, g, coef);
        float gsh[3 * K];
#pragma unroll
        for (int i = 0; i < 3 * K; ++i) gsh[i] = 0.f;
        for (int vi = 0; vi < views.n_views; ++vi) {
            if (!((valid >> vi) & 1u)) continue;
            const DevView& cam = views.v[vi];
            const float dcol_in[3] = {s_dcol[(vi * 3) * nth + tid], s_dcol[(vi * 3 + 1) * nth + tid],
                                      s_dcol[(vi * 3 + 2) * nth + tid]};
            // colour: SH coefficients and viewing direction
            float dx = px - cam.campos[0], dy = py - cam.campos[1], dz = pz - cam.campos[2];
            const float dinv = rsqrtf(dx * dx + dy * dy + dz * dz);
            dx *= dinv; dy *= dinv; dz *= dinv;
            float Y[K];
            sh_basis<DEG>(dx, dy, dz, Y);
            float dcol[3];
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                float acc = 0.5f;
#pragma unroll
                for (int k = 0; k < K; ++k) acc += coef[3 * k + ch] * Y[k];
                dcol[ch] = acc < 0.f ? 0.f : dcol_in[ch];
            }
#pragma unroll
            for (int k = 0; k < K; ++k) {
                gsh[3 * k] += dcol[0] * Y[k];
                gsh[3 * k + 1] += dcol[1] * Y[k];
                gsh[3 * k + 2] += dcol[2] * Y[k];
            }
            if (DEG > 0) {
                float D[K][3];
                sh_basis_grad<DEG>(dx, dy, dz, D);
                float dd[3] = {0.f, 0.f, 0.f};
#pragma unroll
                for (int k = 1; k < K; ++k) {
                    const float w = dcol[0] * coef[3 * k] + dcol[1] * coef[3 * k + 1] + dcol[2] * coef[3 * k + 2];
                    dd[0] += w * D[k][0];
                    dd[1] += w * D[k][1];
                    dd[2] += w * D[k][2];
                }
                const float proj = dd[0] * dx + dd[1] * dy + dd[2] * dz;
                gp[0] += (dd[0] - proj * dx) * dinv;
                gp[1] += (dd[1] - proj * dy) * dinv;
                gp[2] += (dd[2] - proj * dz) * dinv;
            }
        }
        if (d_sh) {
            float* o = d_sh + g * 3 * K;
#pragma unroll
            for (int i = 0; i < 3 * K; ++i) o[i] = accumulate ? o[i] + gsh[i] : gsh[i];
        }
    }
    if (d_means) {
#pragma unroll
        for (int k = 0; k < 3; ++k) d_means[3 * g + k] = accumulate ? d_means[3 * g + k] + (float)gp[k] : (float)gp[k];
    }
    // mask x opacity: gop is dL/d(M sigmoid(logit)) summed over the views, so
    // dL/dM = gop sigmoid(logit) and dL/dlogit = gop M sigmoid'(logit); the
    // compositing's own mask gradient (of records with mask 1) is not used
    const double mval = st.mask_opacity ? (double)masks[g] : 1.0;
    if (d_opacity_logits) {
        const float v = (float)(gop * mval * opac * (1.0 - opac));
        d_opacity_logits[g] = accumulate ? d_opacity_logits[g] + v : v;
    }
    if (dm_acc && d_masks) {
        const float v = (float)(st.mask_opacity ? gop * opac : dm_acc[g]);
        d_masks[g] = accumulate ? d_masks[g] + v : v;
    }
}

}  // namespace

void launch_project_fwd(hipStream_t stream, const mgs_gaussians& g, const ViewSet& views, const DevSettings& st,
                        float* rec, float* depth, float* radius, uint32_t* tiles, uint32_t* flags, uint32_t* rkeys,
                        uint32_t* rvals) {
    if (g.n == 0) return;
    const dim3 grid((unsigned)((g.n + 255) / 256));
    float4* rec4 = reinterpret_cast<float4*>(rec);
#define MGS_PFWD(D)                                                                                                \
    hipLaunchKernelGGL(project_fwd_kernel<D>, grid, dim3(256), 0, stream, g.means, g.log_scales, g.quats,          \
                       g.opacity_logits, g.sh, g.masks, g.n, views, st, rec4, depth, radius, tiles, flags, rkeys, \
                       rvals)
    switch (st.sh_degree) {
        case 0: MGS_PFWD(0); break;
        case 1: MGS_PFWD(1); break;
        case 2: MGS_PFWD(2); break;
        default: MGS_PFWD(3); break;
    }
#undef MGS_PFWD
}

namespace {
template <typename AccT>
void project_bwd_t(hipStream_t stream, const mgs_gaussians& g, const ViewSet& views, const DevSettings& st,
                   const AccT* d_rec, const double* dm_acc, AccT* clear, const mgs_gradients& out,
                   const uint32_t* tiles = nullptr) {
    if (g.n == 0) return;
    const dim3 grid((unsigned)((g.n + 255) / 256));
    const size_t lds = (size_t)views.n_views * 3 * 256 * sizeof(float);  // colour gradients of every view
    float* d_masks = dm_acc ? out.d_masks : nullptr;
    float* rec_out = dm_acc ? out.d_records : nullptr;  // whole path only
#define MGS_PBWD_T(D, A, T)                                                                                       \
    hipLaunchKernelGGL((project_bwd_kernel<D, AccT, A, T>), grid, dim3(256), lds, stream, g.means, g.log_scales,    \
                       g.quats, g.opacity_logits, g.sh, g.masks, g.n, views, st, d_rec, dm_acc, clear, out.d_means, \
                       out.d_log_scales, out.d_quats, out.d_opacity_logits, out.d_sh, d_masks, rec_out, tiles)
#define MGS_PBWD_A(D, A)             \
    if (tiles)                       \
        MGS_PBWD_T(D, A, true);      \
    else                             \
        MGS_PBWD_T(D, A, false)
#define MGS_PBWD(D)              \
    if (out.accumulate) {        \
        MGS_PBWD_A(D, true);     \
    } else {                     \
        MGS_PBWD_A(D, false);    \
    }
    switch (st.sh_degree) {
        case 0: MGS_PBWD(0); break;
        case 1: MGS_PBWD(1); break;
        case 2: MGS_PBWD(2); break;
        default: MGS_PBWD(3); break;
    }
#undef MGS_PBWD
#undef MGS_PBWD_A
#undef MGS_PBWD_T
}
}  // namespace

void launch_record_field(hipStream_t stream, const float* rec, int64_t R, int field, float* out) {
    if (R <= 0) return;
    hipLaunchKernelGGL(record_field_kernel, dim3((unsigned)((R + 255) / 256)), dim3(256), 0, stream, rec, R, field,
                       out);
}

void launch_project_bwd(hipStream_t stream, const mgs_gaussians& g, const ViewSet& views, const DevSettings& st,
                        const float* d_rec, const mgs_gradients& out) {
    project_bwd_t<float>(stream, g, views, st, d_rec, nullptr, nullptr, out);
}

void launch_project_bwd64(hipStream_t stream, const mgs_gaussians& g, const ViewSet& views, const DevSettings& st,
                          double* d_rec, const double* dm_acc, const mgs_gradients& out, const uint32_t* tiles) {
    project_bwd_t<double>(stream, g, views, st, d_rec, dm_acc, nullptr, out, tiles);
}

}  // namespace mgs
