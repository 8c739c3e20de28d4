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
// fixed-order tree over the threads.  `entries`: Gram entries per block partial (gridDim.x).
__global__ void __launch_bounds__(256) k_fr_gram_final(const double *partials, int nb, double *out)
{
    __shared__ double sh[2][256];
    const int e = blockIdx.x, t = threadIdx.x;
    const uint64_t entries = gridDim.x;
    double sx = 0.0, sy = 0.0;
    for (int b = t; b < nb; b += 256) {
        sx += partials[((uint64_t)b * entries + e) * 2];
        sy += partials[((uint64_t)b * entries + e) * 2 + 1];
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

// ---------------------------------------------------------------------------------------
// Two-qubit Kraus sets (a noisy controlled phase, eq. 9 and eq. 14): the same construction over
// quarter-columns.  For qubits (q0, q1) the column v_c splits into four quarters
// h_{c,x}[k] = v_c[k with bit q0 = x & 1, bit q1 = x >> 1], x = 0..3, and
// G = sum_{x,y} (E_a^dagger E_b)[x, y] Gamma4[(x, c), (y, d)] with Gamma4 the Gram matrix of
// the 4r quarter-columns (index a = x * 8 + c, 32 x 32).
// ---------------------------------------------------------------------------------------
constexpr int kFrG2 = 4 * kFrMax;    // quarter-columns

__device__ __forceinline__ uint64_t fr_quad_index(uint64_t k, int lo, int hi, int q0, int q1, int x)
{
    return fr_ins0(fr_ins0(k, lo), hi) | ((uint64_t)(x & 1) << q0) | ((uint64_t)(x >> 1) << q1);
}

static inline int fr2_log_blocks(int n)
{
    // rows per column 2^(n-2); every wave of the matrix-core kernel needs >= 16 of them
    int lb = fr_log_blocks(n);
    const int cap = (n - 2) - 2 - 4;
    if (lb > cap) lb = cap;
    return lb < 0 ? 0 : lb;
}

// Gamma4 on the FP64 matrix cores.  Lane l feeds quarter-column m = l % 16 of block 0 (x = 0, 1)
// and of block 1 (x = 2, 3) for its row (l / 16 of each group of four rows).  The diagonal
// blocks are H^dagger H of their 16 quarter-columns as in k_fr_gram_mfma (three products); the
// block (0, 1) needs four: Re = P0r^T P1r + P0i^T P1i, Im = P0r^T P1i - P0i^T P1r.
template <typename R>
__global__ void __launch_bounds__(256) k_fr_gram2_mfma(const R *V, int n, int r_in, int q0, int q1,
                                                       int log_blocks, double *partials)
{
    __shared__ double red[4][6][256];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15, j = lane >> 4;
    const int x0 = m / kFrMax, c = m % kFrMax;
    const bool live = c < r_in;
    const R *col = V + ((uint64_t)(live ? c : 0) << (n + 1));
    const int lo = q0 < q1 ? q0 : q1, hi = q0 < q1 ? q1 : q0;
    const uint64_t per_block = (1ull << (n - 2)) >> log_blocks;
    const uint64_t per_wave = per_block >> 2;
    const uint64_t begin = (uint64_t)blockIdx.x * per_block + (uint64_t)wave * per_wave;
    fr_d4 z = {0.0, 0.0, 0.0, 0.0};
    fr_d4 d00r = z, d00x = z, d11r = z, d11x = z, d01r = z, d01i = z;
    for (uint64_t p0 = begin; p0 < begin + per_wave; p0 += 16) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const uint64_t k = p0 + 4 * j + t;
            double ar = 0.0, ai = 0.0, br = 0.0, bi = 0.0;
            if (live) {
                const uint64_t ia = fr_quad_index(k, lo, hi, q0, q1, x0);
                const uint64_t ib = fr_quad_index(k, lo, hi, q0, q1, x0 + 2);
                ar = (double)col[2 * ia];
                ai = (double)col[2 * ia + 1];
                br = (double)col[2 * ib];
                bi = (double)col[2 * ib + 1];
            }
            d00r = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, ar, d00r, 0, 0, 0);
            d00r = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, ai, d00r, 0, 0, 0);
            d00x = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, ai, d00x, 0, 0, 0);
            d11r = __builtin_amdgcn_mfma_f64_16x16x4f64(br, br, d11r, 0, 0, 0);
            d11r = __builtin_amdgcn_mfma_f64_16x16x4f64(bi, bi, d11r, 0, 0, 0);
            d11x = __builtin_amdgcn_mfma_f64_16x16x4f64(br, bi, d11x, 0, 0, 0);
            d01r = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, br, d01r, 0, 0, 0);
            d01r = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, bi, d01r, 0, 0, 0);
            d01i = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, bi, d01i, 0, 0, 0);
            d01i = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai, br, d01i, 0, 0, 0);
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int e = (4 * i + j) * 16 + m;
        red[wave][0][e] = d00r[i];
        red[wave][1][e] = d00x[i];
        red[wave][2][e] = d11r[i];
        red[wave][3][e] = d11x[i];
        red[wave][4][e] = d01r[i];
        red[wave][5][e] = d01i[i];
    }
    __syncthreads();
    const int t = threadIdx.x, I = t >> 4, J = t & 15, tt = J * 16 + I;
    auto sum = [&](int a, int e) { return red[0][a][e] + red[1][a][e] + red[2][a][e] + red[3][a][e]; };
    double *o = partials + (uint64_t)blockIdx.x * (kFrG2 * kFrG2) * 2;
    auto put = [&](int a, int b, double re, double im) {
        o[2 * (a * kFrG2 + b)] = re;
        o[2 * (a * kFrG2 + b) + 1] = im;
    };
    put(I, J, sum(0, t), sum(1, t) - sum(1, tt));
    put(16 + I, 16 + J, sum(2, t), sum(3, t) - sum(3, tt));
    put(I, 16 + J, sum(4, t), sum(5, t));
    put(16 + I, J, sum(4, tt), -sum(5, tt));
}

// Small states (fewer than 16 rows per wave): one block, each thread sums its entries over the
// rows directly.
template <typename R>
__global__ void __launch_bounds__(256) k_fr_gram2_small(const R *V, int n, int r_in, int q0, int q1,
                                                        double *partials)
{
    const int lo = q0 < q1 ? q0 : q1, hi = q0 < q1 ? q1 : q0;
    const uint64_t rows = 1ull << (n - 2);
    for (int e = threadIdx.x; e < kFrG2 * kFrG2; e += 256) {
        const int a = e / kFrG2, b = e % kFrG2;
        const int xa = a / kFrMax, ca = a % kFrMax, xb = b / kFrMax, cb = b % kFrMax;
        double sr = 0.0, si = 0.0;
        if (ca < r_in && cb < r_in) {
            const R *pa = V + ((uint64_t)ca << (n + 1)), *pb = V + ((uint64_t)cb << (n + 1));
            for (uint64_t k = 0; k < rows; ++k) {
                const uint64_t ia = fr_quad_index(k, lo, hi, q0, q1, xa);
                const uint64_t ib = fr_quad_index(k, lo, hi, q0, q1, xb);
                const double ar = pa[2 * ia], ai = pa[2 * ia + 1], br = pb[2 * ib], bi = pb[2 * ib + 1];
                sr += ar * br + ai * bi;
                si += ar * bi - ai * br;
            }
        }
        partials[2 * e] = sr;
        partials[2 * e + 1] = si;
    }
}

// coef2: 32 x 32 complex doubles, row (x' * 8 + k'), column (y * 8 + c); one thread per row k
// of the quarter-columns.
template <typename R>
__global__ void __launch_bounds__(256) k_fr_recombine2(R *V, int n, int r_in, int r_out, int q0, int q1,
                                                       const double *coef)
{
    __shared__ R cs[kFrG2 * kFrG2][2];
    for (int v = threadIdx.x; v < kFrG2 * kFrG2; v += 256) {
        cs[v][0] = (R)coef[2 * v];
        cs[v][1] = (R)coef[2 * v + 1];
    }
    __syncthreads();
    const int lo = q0 < q1 ? q0 : q1, hi = q0 < q1 ? q1 : q0;
    const uint64_t rows = 1ull << (n - 2);
    const uint64_t k = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= rows) return;
    uint64_t idx[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) idx[x] = fr_quad_index(k, lo, hi, q0, q1, x);
    R hr[kFrG2], hi_[kFrG2];
#pragma unroll
    for (int a = 0; a < kFrG2; ++a) {
        const int x = a / kFrMax, c = a % kFrMax;
        hr[a] = (R)0;
        hi_[a] = (R)0;
        if (c < r_in) {
            const R *p = V + ((uint64_t)c << (n + 1));
            hr[a] = p[2 * idx[x]];
            hi_[a] = p[2 * idx[x] + 1];
        }
    }
    for (int o = 0; o < kFrG2; ++o) {
        const int xo = o / kFrMax, ko = o % kFrMax;
        if (ko >= r_out) continue;
        R sr = (R)0, si = (R)0;
#pragma unroll
        for (int a = 0; a < kFrG2; ++a) {
            const R cr = cs[o * kFrG2 + a][0], ci = cs[o * kFrG2 + a][1];
            sr += cr * hr[a] - ci * hi_[a];
            si += cr * hi_[a] + ci * hr[a];
        }
        R *p = V + ((uint64_t)ko << (n + 1));
        p[2 * idx[xo]] = sr;
        p[2 * idx[xo] + 1] = si;
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
    const size_t one = ((size_t)1 << fr_log_blocks(n)) * 256 * 2;
    const size_t two = n >= 2 ? ((size_t)1 << fr2_log_blocks(n)) * kFrG2 * kFrG2 * 2 : 0;
    return one > two ? one : two;
}

hipError_t launch_fr_gram2(const void *V, qs_dtype dt, int n, int r, int q0, int q1, double *partials,
                           double *gram_out, hipStream_t st)
{
    const int lb = fr2_log_blocks(n);
    TimedLaunch tl("fr_gram", (double)r * (double)(1ull << n) * amp_bytes(dt), st);
    if ((n - 2) - lb - 2 >= 4) {
        if (dt == QS_C64)
            hipLaunchKernelGGL(k_fr_gram2_mfma<float>, dim3(1u << lb), dim3(256), 0, st, (const float *)V, n, r,
                               q0, q1, lb, partials);
        else
            hipLaunchKernelGGL(k_fr_gram2_mfma<double>, dim3(1u << lb), dim3(256), 0, st, (const double *)V, n,
                               r, q0, q1, lb, partials);
        hipLaunchKernelGGL(k_fr_gram_final, dim3(kFrG2 * kFrG2), dim3(256), 0, st, partials, 1 << lb, gram_out);
    } else {
        if (dt == QS_C64)
            hipLaunchKernelGGL(k_fr_gram2_small<float>, dim3(1), dim3(256), 0, st, (const float *)V, n, r, q0, q1,
                               partials);
        else
            hipLaunchKernelGGL(k_fr_gram2_small<double>, dim3(1), dim3(256), 0, st, (const double *)V, n, r, q0,
                               q1, partials);
        hipLaunchKernelGGL(k_fr_gram_final, dim3(kFrG2 * kFrG2), dim3(256), 0, st, partials, 1, gram_out);
    }
    return hipGetLastError();
}

hipError_t launch_fr_recombine2(void *V, qs_dtype dt, int n, int r_in, int r_out, int q0, int q1,
                                const double *coef_dev, hipStream_t st)
{
    const uint64_t rows = 1ull << (n - 2);
    const unsigned blocks = (unsigned)((rows + 255) / 256);
    TimedLaunch tl("fr_recombine",
                   ((double)r_in + (double)r_out) * (double)(1ull << n) * amp_bytes(dt), st);
    if (dt == QS_C64)
        hipLaunchKernelGGL(k_fr_recombine2<float>, dim3(blocks), dim3(256), 0, st, (float *)V, n, r_in, r_out,
                           q0, q1, coef_dev);
    else
        hipLaunchKernelGGL(k_fr_recombine2<double>, dim3(blocks), dim3(256), 0, st, (double *)V, n, r_in, r_out,
                           q0, q1, coef_dev);
    return hipGetLastError();
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
