// Fixed-rank density matrix kernels (Section 3.2).
//
// rho = sum_c |v_c><v_c| with the columns v_c stored as state vectors.  For a one-qubit Kraus
// set {E_a} on qubit q, W = [E_a v_c] and G = W^dagger W = sum_{x,y} (E_a^dagger E_b)[x, y]
// Gamma[(x, c), (y, d)], where Gamma is the Gram matrix of the 2r half-columns
// h_{c,x}[k] = v_c[k with bit q = x].  The kernels compute Gamma in FP64 in one read of the
// columns, and apply the truncated recombination v'_k[x'] = sum C[(x', k), (y, c)] h_{c,y} in
// one read and one write.
#include "internal.h"

namespace qs {

constexpr int kFrMax = 8;            // columns (rank bound r)
constexpr int kFrG = 2 * kFrMax;     // half-columns
constexpr int kFrChunk = 64;         // pairs staged per LDS chunk

__device__ __forceinline__ uint64_t fr_ins0(uint64_t x, int q)
{
    uint64_t lo = x & ((1ull << q) - 1);
    return ((x ^ lo) << 1) | lo;
}

static inline int fr_log_blocks(int n)
{
    // pairs per slot 2^(n-1); each block takes >= 16 chunks
    int lb = (n - 1) - 10;
    if (lb < 0) lb = 0;
    if (lb > 10) lb = 10;
    return lb;
}

template <typename R>
__global__ void __launch_bounds__(256) k_fr_gram(const R *V, int n, int r_in, int q, int log_blocks,
                                                 double *partials)
{
    __shared__ double2 xs[kFrChunk][kFrG];
    __shared__ double2 red[16][16][16];   // [row group][4x4 block][entry]
    const int tid = threadIdx.x;
    const int blk16 = tid & 15, bi = blk16 >> 2, bj = blk16 & 3, rg = tid >> 4;
    const uint64_t N = 1ull << n;
    const uint64_t pairs = N >> 1;
    const uint64_t per = pairs >> log_blocks;
    const uint64_t begin = (uint64_t)blockIdx.x * per;
    double2 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = make_double2(0.0, 0.0);

    for (uint64_t c0 = begin; c0 < begin + per; c0 += kFrChunk) {
        const uint64_t rows = (begin + per - c0) < (uint64_t)kFrChunk ? (begin + per - c0) : kFrChunk;
        __syncthreads();
        for (int v = tid; v < kFrChunk * kFrG; v += 256) {
            int a = v / kFrChunk, row = v % kFrChunk;
            int x = a / kFrMax, c = a % kFrMax;
            double2 val = make_double2(0.0, 0.0);
            if (c < r_in && (uint64_t)row < rows) {
                uint64_t i = fr_ins0(c0 + row, q) | ((uint64_t)x << q);
                const R *p = V + ((uint64_t)c << (n + 1));
                val = make_double2((double)p[2 * i], (double)p[2 * i + 1]);
            }
            xs[row][a] = val;
        }
        __syncthreads();
        for (int row = rg; row < kFrChunk; row += 16) {
            double2 xi[4], xj[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                xi[k] = xs[row][4 * bi + k];
                xj[k] = xs[row][4 * bj + k];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    // conj(xi) * xj
                    acc[i][j].x += xi[i].x * xj[j].x + xi[i].y * xj[j].y;
                    acc[i][j].y += xi[i].x * xj[j].y - xi[i].y * xj[j].x;
                }
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) red[rg][blk16][4 * i + j] = acc[i][j];
    __syncthreads();
    {
        // thread t owns Gram entry (I, J) = (t >> 4, t & 15)
        const int I = tid >> 4, J = tid & 15;
        const int b = (I >> 2) * 4 + (J >> 2), e = (I & 3) * 4 + (J & 3);
        double sx = 0.0, sy = 0.0;
        for (int g = 0; g < 16; ++g) {
            sx += red[g][b][e].x;
            sy += red[g][b][e].y;
        }
        double *o = partials + ((uint64_t)blockIdx.x * 256 + tid) * 2;
        o[0] = sx;
        o[1] = sy;
    }
}

// The same Gram matrix on the FP64 matrix cores.  Gamma = H^dagger H with H the
// (pairs x 16) matrix of half-columns is a dense contraction over the pairs: with
// H = Hr + i Hi, Re Gamma = Hr^T Hr + Hi^T Hi and Im Gamma = X - X^T with X = Hr^T Hi: three
// real 16 x 16 x 4 products per 4 pairs.  Lane l feeds half-column m = l % 16 of pair k = l / 16 of
// its group as both the A operand (row m, column k) and the B operand (row k, column m);
// accumulator register i of lane l holds row 4 i + l / 16, column l % 16 of the product.  Every wave walks its
// own range of pairs 16 at a time (4 consecutive pairs per lane and half-column), so the main
// loop has no LDS traffic.
typedef double fr_d4 __attribute__((ext_vector_type(4)));

template <typename R>
__global__ void __launch_bounds__(256) k_fr_gram_mfma(const R *V, int n, int r_in, int q, int log_blocks,
                                                      double *partials)
{
    __shared__ double red[4][2][256];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15, j = lane >> 4;
    const int x = m / kFrMax, c = m % kFrMax;
    const bool live = c < r_in;
    const R *col = V + ((uint64_t)(live ? c : 0) << (n + 1));
    const uint64_t per_block = (1ull << (n - 1)) >> log_blocks;
    const uint64_t per_wave = per_block >> 2;
    const uint64_t begin = (uint64_t)blockIdx.x * per_block + (uint64_t)wave * per_wave;
    const uint64_t xbit = (uint64_t)x << q;
    // two independent accumulator pairs alternate, so consecutive products do not wait on
    // each other
    fr_d4 ar0 = {0.0, 0.0, 0.0, 0.0}, ai0 = ar0, ar1 = ar0, ai1 = ar0;
    auto prod = [&](double hr, double hi, fr_d4 &ar, fr_d4 &ai) {
        ar = __builtin_amdgcn_mfma_f64_16x16x4f64(hr, hr, ar, 0, 0, 0);
        ai = __builtin_amdgcn_mfma_f64_16x16x4f64(hr, hi, ai, 0, 0, 0);
        ar = __builtin_amdgcn_mfma_f64_16x16x4f64(hi, hi, ar, 0, 0, 0);
    };
    if (q >= 2) {
        // the lane's 4 consecutive pairs are 4 consecutive amplitudes: one contiguous load
        for (uint64_t p0 = begin; p0 < begin + per_wave; p0 += 16) {
            const uint64_t i = fr_ins0(p0 + 4 * j, q) | xbit;
            double h[8];
            if constexpr (sizeof(R) == 4) {
                float4 u = {0.f, 0.f, 0.f, 0.f}, v = u;
                if (live) {
                    u = *reinterpret_cast<const float4 *>(col + 2 * i);
                    v = *reinterpret_cast<const float4 *>(col + 2 * i + 4);
                }
                h[0] = u.x; h[1] = u.y; h[2] = u.z; h[3] = u.w;
                h[4] = v.x; h[5] = v.y; h[6] = v.z; h[7] = v.w;
            } else {
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    double2 u = live ? *reinterpret_cast<const double2 *>(col + 2 * (i + t)) : double2{0.0, 0.0};
                    h[2 * t] = u.x;
                    h[2 * t + 1] = u.y;
                }
            }
            prod(h[0], h[1], ar0, ai0);
            prod(h[2], h[3], ar1, ai1);
            prod(h[4], h[5], ar0, ai0);
            prod(h[6], h[7], ar1, ai1);
        }
    } else {
        for (uint64_t p0 = begin; p0 < begin + per_wave; p0 += 16) {
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const uint64_t i = fr_ins0(p0 + 4 * j + t, q) | xbit;
                const double hr = live ? (double)col[2 * i] : 0.0;
                const double hi = live ? (double)col[2 * i + 1] : 0.0;
                if (t & 1) prod(hr, hi, ar1, ai1);
                else prod(hr, hi, ar0, ai0);
            }
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        red[wave][0][(4 * i + j) * 16 + m] = ar0[i] + ar1[i];
        red[wave][1][(4 * i + j) * 16 + m] = ai0[i] + ai1[i];
    }
    __syncthreads();
    // Im Gamma = X - X^T with X = Hr^T Hi (the imaginary accumulators hold X)
    const int t = threadIdx.x, tt = (t & 15) * 16 + (t >> 4);
    double sx = red[0][0][t] + red[1][0][t] + red[2][0][t] + red[3][0][t];
    double sy = (red[0][1][t] + red[1][1][t] + red[2][1][t] + red[3][1][t]) -
                (red[0][1][tt] + red[1][1][tt] + red[2][1][tt] + red[3][1][tt]);
    double *o = partials + ((uint64_t)blockIdx.x * 256 + t) * 2;
    o[0] = sx;
    o[1] = sy;
}

// One block per Gram entry: its threads take the blocks' partials in a fixed stride, then a
// fixed-order tree over the threads.
__global__ void __launch_bounds__(256) k_fr_gram_final(const double *partials, int nb, double *out)
{
    __shared__ double sh[2][256];
    const int e = blockIdx.x, t = threadIdx.x;
    double sx = 0.0, sy = 0.0;
    for (int b = t; b < nb; b += 256) {
        sx += partials[((uint64_t)b * 256 + e) * 2];
        sy += partials[((uint64_t)b * 256 + e) * 2 + 1];
    }
    sh[0][t] = sx;
    sh[1][t] = sy;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) {
            sh[0][t] += sh[0][t + s];
            sh[1][t] += sh[1][t + s];
        }
        __syncthreads();
    }
    if (t == 0) {
        out[2 * e] = sh[0][0];
        out[2 * e + 1] = sh[1][0];
    }
}

// coef: 16 x 16 complex doubles, row (x' * 8 + k'), column (y * 8 + c).
template <typename R>
__global__ void __launch_bounds__(256) k_fr_recombine(R *V, int n, int r_in, int r_out, int q,
                                                      const double *coef)
{
    __shared__ R cs[kFrG * kFrG][2];
    for (int v = threadIdx.x; v < kFrG * kFrG; v += 256) {
        cs[v][0] = (R)coef[2 * v];
        cs[v][1] = (R)coef[2 * v + 1];
    }
    __syncthreads();
    const uint64_t pairs = 1ull << (n - 1);
    const uint64_t k = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= pairs) return;
    const uint64_t i0 = fr_ins0(k, q), i1 = i0 | (1ull << q);
    R hr[kFrG], hi[kFrG];
#pragma unroll
    for (int a = 0; a < kFrG; ++a) {
        int x = a / kFrMax, c = a % kFrMax;
        hr[a] = (R)0;
        hi[a] = (R)0;
        if (c < r_in) {
            const R *p = V + ((uint64_t)c << (n + 1));
            uint64_t i = x ? i1 : i0;
            hr[a] = p[2 * i];
            hi[a] = p[2 * i + 1];
        }
    }
    for (int o = 0; o < kFrG; ++o) {
        int xo = o / kFrMax, ko = o % kFrMax;
        if (ko >= r_out) continue;
        R sr = (R)0, si = (R)0;
#pragma unroll
        for (int a = 0; a < kFrG; ++a) {
            R cr = cs[o * kFrG + a][0], ci = cs[o * kFrG + a][1];
            sr += cr * hr[a] - ci * hi[a];
            si += cr * hi[a] + ci * hr[a];
        }
        R *p = V + ((uint64_t)ko << (n + 1));
        uint64_t i = xo ? i1 : i0;
        p[2 * i] = sr;
        p[2 * i + 1] = si;
    }
}

size_t fr_gram_partials_doubles(int n, int r)
{
    (void)r;
    return ((size_t)1 << fr_log_blocks(n)) * 256 * 2;
}

hipError_t launch_fr_gram(const void *V, qs_dtype dt, int n, int r, int q, double *partials,
                          double *gram_out, hipStream_t st)
{
    int lb = fr_log_blocks(n);
    TimedLaunch tl("fr_gram", (double)r * (double)(1ull << n) * amp_bytes(dt), st);
    // matrix-core path: every wave needs a whole number of 16-pair groups
    if ((n - 1) - lb - 2 >= 4) {
        if (dt == QS_C64)
            hipLaunchKernelGGL(k_fr_gram_mfma<float>, dim3(1u << lb), dim3(256), 0, st, (const float *)V, n,
                               r, q, lb, partials);
        else
            hipLaunchKernelGGL(k_fr_gram_mfma<double>, dim3(1u << lb), dim3(256), 0, st, (const double *)V,
                               n, r, q, lb, partials);
    } else if (dt == QS_C64)
        hipLaunchKernelGGL(k_fr_gram<float>, dim3(1u << lb), dim3(256), 0, st, (const float *)V, n,
                           r, q, lb, partials);
    else
        hipLaunchKernelGGL(k_fr_gram<double>, dim3(1u << lb), dim3(256), 0, st, (const double *)V,
                           n, r, q, lb, partials);
    hipLaunchKernelGGL(k_fr_gram_final, dim3(256), dim3(256), 0, st, partials, 1 << lb, gram_out);
    return hipGetLastError();
}

hipError_t launch_fr_recombine(void *V, qs_dtype dt, int n, int r_in, int r_out, int q,
                               const double *coef_dev, hipStream_t st)
{
    uint64_t pairs = 1ull << (n - 1);
    unsigned blocks = (unsigned)((pairs + 255) / 256);
    TimedLaunch tl("fr_recombine",
                   ((double)r_in + (double)r_out) * (double)(1ull << n) * amp_bytes(dt), st);
    if (dt == QS_C64)
        hipLaunchKernelGGL(k_fr_recombine<float>, dim3(blocks), dim3(256), 0, st, (float *)V, n, r_in,
                           r_out, q, coef_dev);
    else
        hipLaunchKernelGGL(k_fr_recombine<double>, dim3(blocks), dim3(256), 0, st, (double *)V, n,
                           r_in, r_out, q, coef_dev);
    return hipGetLastError();
}

}  // namespace qs
