// gfx950 kernels of libqsim: noise draws, the per-(gate, trajectory) noisy-operator table,
// unfused per-gate sweeps over batches of state vectors, and FP64 reductions.
//
// Sweeps are HBM-bound: every dense gate reads and writes each amplitude once.  Threads of a
// block take consecutive 16-byte chunks so that each wave instruction touches one contiguous
// 1 KiB range; a chunk is two complex<float> or one complex<double>.
#include <algorithm>

#include "internal.h"

#include <cmath>

namespace qs {

template <typename R>
struct cx {
    R re, im;
};

template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

template <typename R>
__device__ __forceinline__ cx<R> cfma(cx<R> a, cx<R> b, cx<R> c)  // a * b + c
{
    return {a.re * b.re - a.im * b.im + c.re, a.re * b.im + a.im * b.re + c.im};
}

// Amplitudes per 16-byte vector.
template <typename R>
constexpr int kVec = sizeof(R) == 4 ? 2 : 1;

template <typename R>
__device__ __forceinline__ void vload(const R *psi, uint64_t i, cx<R> *a)
{
    if constexpr (sizeof(R) == 4) {
        float4 v = *reinterpret_cast<const float4 *>(psi + 2 * i);
        a[0] = {v.x, v.y};
        a[1] = {v.z, v.w};
    } else {
        double2 v = *reinterpret_cast<const double2 *>(psi + 2 * i);
        a[0] = {v.x, v.y};
    }
}

template <typename R>
__device__ __forceinline__ void vstore(R *psi, uint64_t i, const cx<R> *a)
{
    if constexpr (sizeof(R) == 4) {
        *reinterpret_cast<float4 *>(psi + 2 * i) = make_float4(a[0].re, a[0].im, a[1].re, a[1].im);
    } else {
        *reinterpret_cast<double2 *>(psi + 2 * i) = make_double2(a[0].re, a[0].im);
    }
}

// Streaming (non-temporal) forms: the sweep reads and writes every line once, so it keeps
// them out of the caches.
typedef float qs_f4 __attribute__((ext_vector_type(4)));
typedef double qs_d2 __attribute__((ext_vector_type(2)));

template <typename R>
__device__ __forceinline__ void vload_nt(const R *psi, uint64_t i, cx<R> *a)
{
    if constexpr (sizeof(R) == 4) {
        qs_f4 v = __builtin_nontemporal_load(reinterpret_cast<const qs_f4 *>(psi + 2 * i));
        a[0] = {v.x, v.y};
        a[1] = {v.z, v.w};
    } else {
        qs_d2 v = __builtin_nontemporal_load(reinterpret_cast<const qs_d2 *>(psi + 2 * i));
        a[0] = {v.x, v.y};
    }
}

template <typename R>
__device__ __forceinline__ void vstore_nt(R *psi, uint64_t i, const cx<R> *a)
{
    if constexpr (sizeof(R) == 4) {
        qs_f4 v = {a[0].re, a[0].im, a[1].re, a[1].im};
        __builtin_nontemporal_store(v, reinterpret_cast<qs_f4 *>(psi + 2 * i));
    } else {
        qs_d2 v = {a[0].re, a[0].im};
        __builtin_nontemporal_store(v, reinterpret_cast<qs_d2 *>(psi + 2 * i));
    }
}

template <typename R>
__device__ __forceinline__ cx<R> sload(const R *psi, uint64_t i)
{
    return {psi[2 * i], psi[2 * i + 1]};
}

template <typename R>
__device__ __forceinline__ void sstore(R *psi, uint64_t i, cx<R> a)
{
    psi[2 * i] = a.re;
    psi[2 * i + 1] = a.im;
}

// Insert a 0 bit at position q of x.
__device__ __forceinline__ uint64_t ins0(uint64_t x, int q)
{
    uint64_t lo = x & ((1ull << q) - 1);
    return ((x ^ lo) << 1) | lo;
}

template <typename R>
__device__ __forceinline__ cx<R> tab_c(const double *t, int k)
{
    return {(R)t[2 * k], (R)t[2 * k + 1]};
}

// ---------------------------------------------------------------------------------------
// Noise: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and the Box-Muller cosine branch.
// The transform uses only correctly rounded IEEE operations with contraction disabled, so a
// deviate is a fixed function of the four counter words.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
        uint32_t hi0 = __umulhi(m0, c.x), lo0 = m0 * c.x;
        uint32_t hi1 = __umulhi(m1, c.z), lo1 = m1 * c.z;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// ln x for positive normal x: x = m 2^k, m in [1/sqrt2, sqrt2), ln m = 2 atanh((m-1)/(m+1))
// summed as its odd power series to s^23.
__device__ double dev_ln(double x)
{
#pragma clang fp contract(off)
    const double ln2_hi = 0x1.62e42fee00000p-1;
    const double ln2_lo = 0x1.a39ef35793c76p-33;
    const double sqrt2 = 0x1.6a09e667f3bcdp+0;
    unsigned long long b = (unsigned long long)__double_as_longlong(x);
    int k = (int)((b >> 52) & 0x7ffull) - 1023;
    double m = __longlong_as_double((long long)((b & 0x000fffffffffffffull) | 0x3ff0000000000000ull));
    if (m > sqrt2) {
        m = m * 0.5;
        k = k + 1;
    }
    double s = (m - 1.0) / (m + 1.0);
    double s2 = s * s;
    double t = 1.0 / 23.0;
    t = t * s2 + 1.0 / 21.0;
    t = t * s2 + 1.0 / 19.0;
    t = t * s2 + 1.0 / 17.0;
    t = t * s2 + 1.0 / 15.0;
    t = t * s2 + 1.0 / 13.0;
    t = t * s2 + 1.0 / 11.0;
    t = t * s2 + 1.0 / 9.0;
    t = t * s2 + 1.0 / 7.0;
    t = t * s2 + 1.0 / 5.0;
    t = t * s2 + 1.0 / 3.0;
    t = t * s2 + 1.0;
    double kd = (double)k;
    return kd * ln2_hi + (kd * ln2_lo + 2.0 * s * t);
}

// cos x and sin x on [0, pi/4] from their Taylor series (to x^20 and x^19).
__device__ double dev_cos_series(double x)
{
#pragma clang fp contract(off)
    double z = x * x;
    double t = 1.0 / 2432902008176640000.0;
    t = t * z - 1.0 / 6402373705728000.0;
    t = t * z + 1.0 / 20922789888000.0;
    t = t * z - 1.0 / 87178291200.0;
    t = t * z + 1.0 / 479001600.0;
    t = t * z - 1.0 / 3628800.0;
    t = t * z + 1.0 / 40320.0;
    t = t * z - 1.0 / 720.0;
    t = t * z + 1.0 / 24.0;
    t = t * z - 1.0 / 2.0;
    return t * z + 1.0;
}

__device__ double dev_sin_series(double x)
{
#pragma clang fp contract(off)
    double z = x * x;
    double t = -1.0 / 121645100408832000.0;
    t = t * z + 1.0 / 355687428096000.0;
    t = t * z - 1.0 / 1307674368000.0;
    t = t * z + 1.0 / 6227020800.0;
    t = t * z - 1.0 / 39916800.0;
    t = t * z + 1.0 / 362880.0;
    t = t * z - 1.0 / 5040.0;
    t = t * z + 1.0 / 120.0;
    t = t * z - 1.0 / 6.0;
    return x + x * (t * z);
}

// cos(2 pi u), u in [0, 1) a multiple of 2^-53: symmetric reduction to [0, pi/4].
__device__ double dev_cos_2pi(double u)
{
#pragma clang fp contract(off)
    const double two_pi = 0x1.921fb54442d18p+2;
    double v = u >= 0.5 ? 1.0 - u : u;
    if (v <= 0.125) return dev_cos_series(two_pi * v);
    if (v <= 0.375) return dev_sin_series(two_pi * (0.25 - v));
    return -dev_cos_series(two_pi * (0.5 - v));
}

__device__ double dev_normal(uint64_t seed, uint32_t site, uint32_t traj, uint32_t stream,
                             uint32_t request)
{
#pragma clang fp contract(off)
    uint4 w = philox4x32_10(make_uint4(site, traj, stream, request), (uint32_t)seed,
                            (uint32_t)(seed >> 32));
    unsigned long long a = ((((unsigned long long)w.x) << 32) | w.y) >> 11;
    unsigned long long b = ((((unsigned long long)w.z) << 32) | w.w) >> 11;
    double u1 = ((double)a + 1.0) * 0x1.0p-53;
    double u2 = (double)b * 0x1.0p-53;
    return __builtin_sqrt(-2.0 * dev_ln(u1)) * dev_cos_2pi(u2);
}

__global__ void k_noise_draw(uint64_t seed, uint32_t request, uint32_t stream,
                             const uint32_t *sites, int n_sites, uint32_t traj_base, int n_traj,
                             double *out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_sites * n_traj) return;
    int t = (int)(i / n_sites), s = (int)(i % n_sites);
    out[i] = dev_normal(seed, sites[s], traj_base + (uint32_t)t, stream, request);
}

// The operator gate G applies in slot s, written to o[0..7].  U1: U V(e xi) (eq. 1) as a
// complex 2x2, products in FP64; CP: exp(-i (theta + e xi)) in the first two doubles.
__device__ void noisy_operator(const qs_gate &G, int s, const NoiseArgs &na, double *o)
{
    double e = 0.0;
    if (s >= na.first_noisy_slot) e = na.e_dev ? na.e_dev[s] : na.e;
    uint32_t traj = na.traj_base + (uint32_t)(s - na.first_noisy_slot);
    if (G.kind == QS_G_U1) {
        double u[8];
        for (int k = 0; k < 8; ++k) u[k] = G.m[k];
        if (e != 0.0 && G.noise == QS_NOISE_ROT) {
            double xi = dev_normal(na.seed, G.site, traj, 0u, na.request);
            double sn, cs;
            sincos(e * xi, &sn, &cs);
            // V = [[cs, sn], [-sn, cs]] is real: (U V)_{r0} = U_r0 cs - U_r1 sn, (U V)_{r1} = U_r0 sn + U_r1 cs
            for (int r = 0; r < 2; ++r) {
                double a_re = u[4 * r], a_im = u[4 * r + 1], b_re = u[4 * r + 2], b_im = u[4 * r + 3];
                o[4 * r + 0] = a_re * cs - b_re * sn;
                o[4 * r + 1] = a_im * cs - b_im * sn;
                o[4 * r + 2] = a_re * sn + b_re * cs;
                o[4 * r + 3] = a_im * sn + b_im * cs;
            }
        } else {
            for (int k = 0; k < 8; ++k) o[k] = u[k];
        }
    } else if (G.kind == QS_G_CP) {
        double ang = G.theta;
        if (e != 0.0 && G.noise == QS_NOISE_PHASE)
            ang += e * dev_normal(na.seed, G.site, traj, 0u, na.request);
        double sn, cs;
        sincos(ang, &sn, &cs);
        o[0] = cs;
        o[1] = -sn;
        for (int k = 2; k < 8; ++k) o[k] = 0.0;
    } else if (G.kind == QS_G_DIAG) {
        // the pattern's factor (noiseless)
        o[0] = G.m[0];
        o[1] = G.m[1];
        for (int k = 2; k < 8; ++k) o[k] = 0.0;
    } else {
        for (int k = 0; k < 8; ++k) o[k] = 0.0;
    }
}

// tab[(g * S + s) * 8 ..] = operator of gate g in slot s.
__global__ void k_noise_table(const qs_gate *gates, int n_gates, int S, NoiseArgs na, double *tab)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_gates * S) return;
    if (na.dyn) {
        na.seed = na.dyn->seed;
        na.request = na.dyn->request;
        na.traj_base = na.dyn->traj_base;
    }
    int g = (int)(i / S), s = (int)(i % S);
    noisy_operator(gates[g], s, na, tab + i * 8);
}

__global__ void k_noise_one(qs_gate G, int S, NoiseArgs na, double *tab)
{
    int s = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (s >= S) return;
    noisy_operator(G, s, na, tab + (int64_t)s * 8);
}

// ---------------------------------------------------------------------------------------
// Basis initialisation: every slot <- |index>.
// ---------------------------------------------------------------------------------------
template <typename R>
__global__ void k_init_basis(R *psi, int n, uint64_t total_vec, uint64_t index, const RunParams *dyn)
{
    if (dyn) index = (uint64_t)dyn->init;
    constexpr int VEC = kVec<R>;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < total_vec; v += stride) {
        uint64_t i = v * VEC;                    // global amplitude index (slot-major)
        uint64_t in_slot = i & ((1ull << n) - 1);
        cx<R> a[VEC];
#pragma unroll
        for (int k = 0; k < VEC; ++k) a[k] = {(R)((in_slot + k) == index ? 1 : 0), (R)0};
        vstore(psi, i, a);
    }
}

// ---------------------------------------------------------------------------------------
// Dense one-qubit sweep: (psi_i0, psi_i1) <- M (psi_i0, psi_i1), i1 = i0 + 2^q (Section 2).
// MODE 0: q >= log2(vec): a thread takes a 16-byte chunk at i0 and the matching chunk at i1.
// MODE 1: (complex<float>, q = 0): the pair is one 16-byte chunk.
// Items per slot are a power of two; each thread handles U items 256 apart.
// ---------------------------------------------------------------------------------------
template <typename R, int MODE, int U>
__global__ void __launch_bounds__(256) k_u1(R *psi, int n, int q, const double *tab_row,
                                            int log_items, uint64_t total)
{
  for (uint64_t blk = blockIdx.x; blk * (256 * U) < total; blk += gridDim.x) {
    constexpr int VEC = kVec<R>;
    const uint64_t base_item = blk * (256 * U) + threadIdx.x;
    cx<R> a0[U][VEC], a1[U][VEC];
    uint64_t i0s[U];
    int slots[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        uint64_t it = base_item + (uint64_t)u * 256;
        slots[u] = -1;
        if (it >= total) continue;
        int slot = (int)(it >> log_items);
        uint64_t c = it & ((1ull << log_items) - 1);
        R *p = psi + ((uint64_t)slot << (n + 1));
        slots[u] = slot;
        if constexpr (MODE == 0) {
            uint64_t i0 = ins0(c * VEC, q);
            i0s[u] = i0;
            // streaming accesses pay off when the two streams are at least 4 amplitudes apart
            if (q >= 2) {
                vload_nt(p, i0, a0[u]);
                vload_nt(p, i0 | (1ull << q), a1[u]);
            } else {
                vload(p, i0, a0[u]);
                vload(p, i0 | (1ull << q), a1[u]);
            }
        } else {
            i0s[u] = c * 2;
            cx<R> t[2];
            vload_nt(p, c * 2, t);
            a0[u][0] = t[0];
            a1[u][0] = t[1];
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if (slots[u] < 0) continue;
        const double *t = tab_row + (uint64_t)slots[u] * 8;
        cx<R> m00 = tab_c<R>(t, 0), m01 = tab_c<R>(t, 1), m10 = tab_c<R>(t, 2), m11 = tab_c<R>(t, 3);
        R *p = psi + ((uint64_t)slots[u] << (n + 1));
        constexpr int NP = MODE == 0 ? VEC : 1;
        cx<R> b0[VEC], b1[VEC];
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            b0[k] = cfma(m01, a1[u][k], cmul(m00, a0[u][k]));
            b1[k] = cfma(m11, a1[u][k], cmul(m10, a0[u][k]));
        }
        if constexpr (MODE == 0) {
            if (q >= 2) {
                vstore_nt(p, i0s[u], b0);
                vstore_nt(p, i0s[u] | (1ull << q), b1);
            } else {
                vstore(p, i0s[u], b0);
                vstore(p, i0s[u] | (1ull << q), b1);
            }
        } else {
            cx<R> t2[2] = {b0[0], b1[0]};
            vstore_nt(p, i0s[u], t2);
        }
    }
  }
}

// Dense one-qubit sweep with the target among the index bits that a wavefront's 64 lanes span:
// every lane loads its own 16-byte vector (consecutive lanes hold consecutive vectors, so each
// access of a wave is one contiguous 1 KiB) and takes its pair partner from lane l ^ 2^LB with a
// cross-lane permute, LB = q for complex<double> (one amplitude per vector) and q - 1 for
// complex<float> (two).  Each lane then forms its own half of the pair update: with target bit
// 0, m00 a + m01 partner; with 1, m11 a + m10 partner.  Items (vectors) per slot are a multiple
// of 256 U, so every lane of a wave takes part in each permute.
template <typename R, int U>
__global__ void __launch_bounds__(256) k_u1_lane(R *psi, int n, int lb, const double *tab_row, int log_items,
                                                 uint64_t total)
{
  constexpr int VEC = kVec<R>;
  const int lmask = 1 << lb;
  for (uint64_t blk = blockIdx.x; blk * (256 * U) < total; blk += gridDim.x) {
    const uint64_t base_item = blk * (256 * U) + threadIdx.x;
    cx<R> a[U][VEC];
    int slots[U];
    uint64_t cs[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const uint64_t it = base_item + (uint64_t)u * 256;
        slots[u] = (int)(it >> log_items);
        cs[u] = it & ((1ull << log_items) - 1);
        vload_nt(psi + ((uint64_t)slots[u] << (n + 1)), cs[u] * VEC, a[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const double *t = tab_row + (uint64_t)slots[u] * 8;
        const bool one = (cs[u] >> lb) & 1;
        const cx<R> ca = tab_c<R>(t, one ? 3 : 0), cp = tab_c<R>(t, one ? 2 : 1);
        cx<R> b[VEC];
#pragma unroll
        for (int k = 0; k < VEC; ++k) {
            const cx<R> pr = {__shfl_xor(a[u][k].re, lmask), __shfl_xor(a[u][k].im, lmask)};
            b[k] = cfma(cp, pr, cmul(ca, a[u][k]));
        }
        vstore_nt(psi + ((uint64_t)slots[u] << (n + 1)), cs[u] * VEC, b);
    }
  }
}

// Generic one-amplitude-pair-per-thread fallback for small states.
template <typename R>
__global__ void k_u1_small(R *psi, int n, int q, const double *tab_row, uint64_t total)
{
  for (uint64_t it = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; it < total;
       it += (uint64_t)gridDim.x * blockDim.x) {
    int slot = (int)(it >> (n - 1));
    uint64_t c = it & ((1ull << (n - 1)) - 1);
    R *p = psi + ((uint64_t)slot << (n + 1));
    const double *t = tab_row + (uint64_t)slot * 8;
    cx<R> m00 = tab_c<R>(t, 0), m01 = tab_c<R>(t, 1), m10 = tab_c<R>(t, 2), m11 = tab_c<R>(t, 3);
    uint64_t i0 = ins0(c, q), i1 = i0 | (1ull << q);
    cx<R> a0 = sload(p, i0), a1 = sload(p, i1);
    sstore(p, i0, cfma(m01, a1, cmul(m00, a0)));
    sstore(p, i1, cfma(m11, a1, cmul(m10, a0)));
  }
}

// ---------------------------------------------------------------------------------------
// Two-qubit sweeps over the N/4 index groups with bits (lo, hi) fixed.
// KIND 0: controlled phase -- the |11> amplitude times the slot's phase (eq. 2).
// KIND 1: SWAP (01 <-> 10).  KIND 2: CNOT (control qa, target qb).  KIND 3: dense 4x4.
// V amplitudes per chunk (V = vec when lo >= log2 vec, else 1).
// ---------------------------------------------------------------------------------------
struct M32 {
    double v[32];
};

template <typename R, int KIND, int V>
__global__ void __launch_bounds__(256) k_2q(R *psi, int n, int qa, int qb, const double *tab_row,
                                            M32 m32, int log_items, uint64_t total)
{
  for (uint64_t it = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; it < total;
       it += (uint64_t)gridDim.x * blockDim.x) {
    const int lo = qa < qb ? qa : qb, hi = qa < qb ? qb : qa;
    int slot = (int)(it >> log_items);
    uint64_t c = it & ((1ull << log_items) - 1);
    R *p = psi + ((uint64_t)slot << (n + 1));
    uint64_t base = ins0(ins0(c * V, lo), hi);
    const uint64_t ba = 1ull << qa, bb = 1ull << qb;
    // 16-byte vectors (two complex<float> or one complex<double>); streaming accesses for the
    // phase and dense kinds when the runs of contiguous amplitudes are at least 4 long, for the
    // permutations when they are at least 64 long (at n = 28, SWAP and CNOT on high pairs: 62-72%
    // -> 77-79% of HBM; with runs of 4 they measured slower with them)
    const bool nt = (KIND == 0 || KIND == 3) ? lo >= 2 : lo >= 6;
    auto ld = [&](uint64_t i, cx<R> *a) {
        if constexpr (V == kVec<R>) {
            if (nt) vload_nt(p, i, a);
            else vload(p, i, a);
        } else {
            a[0] = sload(p, i);
        }
    };
    auto st = [&](uint64_t i, const cx<R> *a) {
        if constexpr (V == kVec<R>) {
            if (nt) vstore_nt(p, i, a);
            else vstore(p, i, a);
        } else {
            sstore(p, i, a[0]);
        }
    };
    if constexpr (KIND == 0) {
        const double *t = tab_row + (uint64_t)slot * 8;
        cx<R> ph = tab_c<R>(t, 0);
        cx<R> a[V];
        ld(base | ba | bb, a);
#pragma unroll
        for (int k = 0; k < V; ++k) a[k] = cmul(ph, a[k]);
        st(base | ba | bb, a);
    } else if constexpr (KIND == 1 || KIND == 2) {
        uint64_t x = KIND == 1 ? (base | ba) : (base | ba);
        uint64_t y = KIND == 1 ? (base | bb) : (base | ba | bb);
        cx<R> a[V], b[V];
        ld(x, a);
        ld(y, b);
        st(x, b);
        st(y, a);
    } else {
        cx<R> a[4][V];
        uint64_t idx[4] = {base, base | ba, base | bb, base | ba | bb};
#pragma unroll
        for (int r = 0; r < 4; ++r) ld(idx[r], a[r]);
        cx<R> m[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) m[k] = {(R)m32.v[2 * k], (R)m32.v[2 * k + 1]};
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            cx<R> o[V];
#pragma unroll
            for (int k = 0; k < V; ++k) {
                cx<R> s = cmul(m[4 * r], a[0][k]);
                s = cfma(m[4 * r + 1], a[1][k], s);
                s = cfma(m[4 * r + 2], a[2][k], s);
                s = cfma(m[4 * r + 3], a[3][k], s);
                o[k] = s;
            }
            st(idx[r], o);
        }
    }
  }
}

// Dense two-qubit sweep with the lower qubit among a wave's lane bits and the upper one above
// the vectors a wave spans: each lane loads its vector in both halves of the upper qubit (two
// contiguous 1 KiB accesses per wave), takes the partner lane's two vectors (lane l ^ 2^LB,
// LB = lower qubit - log2(amplitudes per vector)) with cross-lane permutes, and forms the two
// outputs of its own lower-qubit value b: y(b, h) = sum over (b', h') of
// m[b + 2h][b' + 2h'] x(b', h') (the host orders m with the lower qubit as the low local bit).
// Items per slot (vectors with the upper qubit clear) are a multiple of 256, so every lane
// takes part in each permute.
template <typename R>
__global__ void __launch_bounds__(256) k_2q_lane(R *psi, int n, int lb, int hb, M32 m32, int log_items,
                                                 uint64_t total)
{
  constexpr int VEC = kVec<R>;
  const int lmask = 1 << lb;
  cx<R> m[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) m[k] = {(R)m32.v[2 * k], (R)m32.v[2 * k + 1]};
  for (uint64_t it = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; it < total;
       it += (uint64_t)gridDim.x * blockDim.x) {
    const int slot = (int)(it >> log_items);
    const uint64_t c = it & ((1ull << log_items) - 1);
    const uint64_t v0 = ins0(c, hb), v1 = v0 | (1ull << hb);
    R *p = psi + ((uint64_t)slot << (n + 1));
    cx<R> A[VEC], B[VEC];
    vload_nt(p, v0 * VEC, A);
    vload_nt(p, v1 * VEC, B);
    const bool b = (c >> lb) & 1;
    // rows b (upper 0) and b + 2 (upper 1); columns: own lower value, partner's, in both halves
    const cx<R> k00 = b ? m[5] : m[0], k01 = b ? m[4] : m[1], k02 = b ? m[7] : m[2], k03 = b ? m[6] : m[3];
    const cx<R> k10 = b ? m[13] : m[8], k11 = b ? m[12] : m[9], k12 = b ? m[15] : m[10], k13 = b ? m[14] : m[11];
    cx<R> Y0[VEC], Y1[VEC];
#pragma unroll
    for (int k = 0; k < VEC; ++k) {
        const cx<R> Ap = {__shfl_xor(A[k].re, lmask), __shfl_xor(A[k].im, lmask)};
        const cx<R> Bp = {__shfl_xor(B[k].re, lmask), __shfl_xor(B[k].im, lmask)};
        Y0[k] = cfma(k03, Bp, cfma(k02, B[k], cfma(k01, Ap, cmul(k00, A[k]))));
        Y1[k] = cfma(k13, Bp, cfma(k12, B[k], cfma(k11, Ap, cmul(k10, A[k]))));
    }
    vstore_nt(p, v0 * VEC, Y0);
    vstore_nt(p, v1 * VEC, Y1);
  }
}

// Sign flip of every amplitude i with (i & mask) == value: the free bits of ~mask are
// enumerated by depositing the item index into them.
template <typename R>
__global__ void k_flip(R *psi, int n, uint64_t mask, uint64_t value, int free_bits,
                       uint64_t total)
{
  for (uint64_t it = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; it < total;
       it += (uint64_t)gridDim.x * blockDim.x) {
    int slot = (int)(it >> free_bits);
    uint64_t c = it & ((1ull << free_bits) - 1);
    uint64_t i = value;
    int b = 0;
    for (int q = 0; q < n; ++q) {
        if (mask & (1ull << q)) continue;
        if (c & (1ull << b)) i |= 1ull << q;
        ++b;
    }
    R *p = psi + ((uint64_t)slot << (n + 1));
    p[2 * i] = -p[2 * i];
    p[2 * i + 1] = -p[2 * i + 1];
  }
}

// The same enumeration, multiplying every selected amplitude by one complex factor (the
// averaged controlled phase on vec(rho)).
template <typename R>
__global__ void k_scale_pattern(R *psi, int n, uint64_t mask, uint64_t value, int free_bits,
                                uint64_t total, double fre, double fim)
{
  const R cr = (R)fre, ci = (R)fim;
  for (uint64_t it = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; it < total;
       it += (uint64_t)gridDim.x * blockDim.x) {
    int slot = (int)(it >> free_bits);
    uint64_t c = it & ((1ull << free_bits) - 1);
    uint64_t i = value;
    int b = 0;
    for (int q = 0; q < n; ++q) {
        if (mask & (1ull << q)) continue;
        if (c & (1ull << b)) i |= 1ull << q;
        ++b;
    }
    R *p = psi + ((uint64_t)slot << (n + 1));
    const R ar = p[2 * i], ai = p[2 * i + 1];
    p[2 * i] = cr * ar - ci * ai;
    p[2 * i + 1] = cr * ai + ci * ar;
  }
}

// ---------------------------------------------------------------------------------------
// FP64 reductions.  Stage 1: each block sums a fixed contiguous range in a fixed order
// (thread-strided, then an LDS tree); stage 2: one block per slot sums the block partials in
// a fixed order.  Results are bitwise reproducible for a given launch shape.
// ---------------------------------------------------------------------------------------
constexpr int kRedThreads = 256;

__device__ __forceinline__ void block_sum(double *sh, double (&v)[4], int nv)
{
    const int t = threadIdx.x;
    for (int k = 0; k < nv; ++k) sh[k * kRedThreads + t] = v[k];
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if (t < s)
            for (int k = 0; k < nv; ++k) sh[k * kRedThreads + t] += sh[k * kRedThreads + t + s];
        __syncthreads();
    }
    for (int k = 0; k < nv; ++k) v[k] = sh[k * kRedThreads];
}

static inline int red_log_blocks(int n)
{
    // blocks per slot: enough to fill the chip for one slot, at least 2^11 amplitudes each
    int lb = n - 11;
    if (lb < 0) lb = 0;
    if (lb > 9) lb = 9;
    return lb;
}

template <typename R>
__global__ void __launch_bounds__(kRedThreads) k_overlap_partial(const R *ref, const R *psi, int n,
                                                                 int log_blocks, double *partials)
{
    __shared__ double sh[3 * kRedThreads];
    // chunk-major order: the blocks of every slot for one chunk run together, so the
    // reference chunk is read from HBM once and from the caches by the other slots
    const int S = (int)(gridDim.x >> log_blocks);
    const int slot = (int)(blockIdx.x % (unsigned)S);
    const uint64_t blk = blockIdx.x / (unsigned)S;
    const uint64_t per = 1ull << (n - log_blocks);
    const R *p = psi + ((uint64_t)slot << (n + 1));
    double v[4] = {0, 0, 0, 0};
    constexpr int VEC = kVec<R>;
    const uint64_t begin = blk * per;
    if (per >= (uint64_t)VEC * kRedThreads) {
        for (uint64_t i = begin + (uint64_t)threadIdx.x * VEC; i < begin + per; i += (uint64_t)VEC * kRedThreads) {
            cx<R> a[VEC], b[VEC];
            vload(ref, i, a);
            vload_nt(p, i, b);
#pragma unroll
            for (int k = 0; k < VEC; ++k) {
                double ar = a[k].re, ai = a[k].im, br = b[k].re, bi = b[k].im;
                v[0] += ar * br + ai * bi;
                v[1] += ar * bi - ai * br;
                v[2] += br * br + bi * bi;
            }
        }
    } else {
        for (uint64_t i = begin + threadIdx.x; i < begin + per; i += kRedThreads) {
            cx<R> a = sload(ref, i), b = sload(p, i);
            double ar = a.re, ai = a.im, br = b.re, bi = b.im;
            v[0] += ar * br + ai * bi;
            v[1] += ar * bi - ai * br;
            v[2] += br * br + bi * bi;
        }
    }
    block_sum(sh, v, 3);
    if (threadIdx.x == 0) {
        double *o = partials + ((uint64_t)slot << log_blocks | blk) * 3;
        o[0] = v[0];
        o[1] = v[1];
        o[2] = v[2];
    }
}

template <typename R>
__global__ void __launch_bounds__(kRedThreads) k_overlap_final(const R *psi, int n, int log_blocks,
                                                               int64_t marked, const double *partials,
                                                               double *out, const RunParams *dyn)
{
    __shared__ double sh[3 * kRedThreads];
    if (dyn) marked = dyn->marked;
    const int slot = blockIdx.x;
    const int nb = 1 << log_blocks;
    double v[4] = {0, 0, 0, 0};
    for (int b = threadIdx.x; b < nb; b += kRedThreads) {
        const double *q = partials + ((uint64_t)slot * nb + b) * 3;
        v[0] += q[0];
        v[1] += q[1];
        v[2] += q[2];
    }
    block_sum(sh, v, 3);
    if (threadIdx.x == 0) {
        double *o = out + (uint64_t)slot * 5;
        o[0] = v[0];
        o[1] = v[1];
        o[2] = v[2];
        if (marked >= 0) {
            const R *p = psi + ((uint64_t)slot << (n + 1));
            o[3] = (double)p[2 * marked];
            o[4] = (double)p[2 * marked + 1];
        } else {
            o[3] = 0.0;
            o[4] = 0.0;
        }
    }
}

// <psi|rho|psi> = sum_ij conj(psi_i) rho_ij psi_j and Tr rho over vec(rho), rho_ij at i 2^n + j.
template <typename R>
__global__ void __launch_bounds__(kRedThreads) k_dm_expect_partial(const R *rho, const R *psi, int n,
                                                                   int log_blocks, double *partials)
{
    __shared__ double sh[4 * kRedThreads];
    const uint64_t per = 1ull << (2 * n - log_blocks);
    const uint64_t begin = (uint64_t)blockIdx.x * per;
    const uint64_t jmask = (1ull << n) - 1;
    double v[4] = {0, 0, 0, 0};
    for (uint64_t idx = begin + threadIdx.x; idx < begin + per; idx += kRedThreads) {
        uint64_t i = idx >> n, j = idx & jmask;
        cx<R> r = sload(rho, idx), pi = sload(psi, i), pj = sload(psi, j);
        double rr = r.re, ri = r.im;
        // conj(pi) * r * pj
        double tr = (double)pi.re * rr + (double)pi.im * ri;
        double ti = (double)pi.re * ri - (double)pi.im * rr;
        v[0] += tr * (double)pj.re - ti * (double)pj.im;
        v[1] += tr * (double)pj.im + ti * (double)pj.re;
        if (i == j) {
            v[2] += rr;
            v[3] += ri;
        }
    }
    block_sum(sh, v, 4);
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; ++k) partials[(uint64_t)blockIdx.x * 4 + k] = v[k];
}

__global__ void __launch_bounds__(kRedThreads) k_sum4_final(const double *partials, int nb, double *out)
{
    __shared__ double sh[4 * kRedThreads];
    double v[4] = {0, 0, 0, 0};
    for (int b = threadIdx.x; b < nb; b += kRedThreads)
        for (int k = 0; k < 4; ++k) v[k] += partials[(uint64_t)b * 4 + k];
    block_sum(sh, v, 4);
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; ++k) out[k] = v[k];
}

__global__ void k_copy(float4 *dst, const float4 *src, uint64_t n16)
{
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (; i < n16; i += stride) dst[i] = src[i];
}

// ---------------------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------------------
// Grid size for `items` work items, `per_block` per block.  AMD GPUs allow fewer than 2^32
// work items per grid dimension, so large sweeps cap the grid and loop (grid-stride).
static inline unsigned blocks_for(uint64_t items, unsigned per_block)
{
    uint64_t b = (items + per_block - 1) / per_block;
    const uint64_t cap = (1ull << 31) / 1024;    // 2^21 blocks of <= 1024 work items
    return (unsigned)(b < cap ? b : cap);
}

hipError_t launch_noise_table(const qs_gate *gates_dev, int n_gates, int S, NoiseArgs na,
                              double *tab, hipStream_t st)
{
    uint64_t tot = (uint64_t)n_gates * S;
    if (tot == 0) return hipSuccess;
    TimedLaunch tl("noise", (double)tot * 64.0, st);
    hipLaunchKernelGGL(k_noise_table, dim3(blocks_for(tot, 128)), dim3(128), 0, st, gates_dev,
                       n_gates, S, na, tab);
    return hipGetLastError();
}

hipError_t launch_noise_one(const qs_gate &g, int S, NoiseArgs na, double *tab, hipStream_t st)
{
    TimedLaunch tl("noise", (double)S * 64.0, st);
    hipLaunchKernelGGL(k_noise_one, dim3((S + 127) / 128), dim3(128), 0, st, g, S, na, tab);
    return hipGetLastError();
}

hipError_t launch_noise_draw(uint64_t seed, uint32_t request, uint32_t stream,
                             const uint32_t *sites, int n_sites, uint32_t traj_base, int n_traj,
                             double *out, hipStream_t st)
{
    uint64_t tot = (uint64_t)n_sites * n_traj;
    if (tot == 0) return hipSuccess;
    hipLaunchKernelGGL(k_noise_draw, dim3(blocks_for(tot, 128)), dim3(128), 0, st, seed, request,
                       stream, sites, n_sites, traj_base, n_traj, out);
    return hipGetLastError();
}

hipError_t launch_init_basis(void *psi, qs_dtype dt, int n, int S, uint64_t index, hipStream_t st,
                             const RunParams *dyn)
{
    uint64_t amps = (uint64_t)S << n;
    TimedLaunch tl("init", (double)amps * amp_bytes(dt), st);
    if (dt == QS_C64) {
        uint64_t tv = amps / 2;
        if (n == 0) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_init_basis<float>, dim3(blocks_for(tv, 256)), dim3(256), 0, st,
                           (float *)psi, n, tv, index, dyn);
    } else {
        hipLaunchKernelGGL(k_init_basis<double>, dim3(blocks_for(amps, 256)), dim3(256), 0, st,
                           (double *)psi, n, amps, index, dyn);
    }
    return hipGetLastError();
}

// Target bits below which the one-qubit sweep exchanges pair partners between lanes (of the
// six lane bits of a wave's vectors).
#ifndef QS_LANE_TARGET_BITS
#define QS_LANE_TARGET_BITS 6
#endif
constexpr int kLaneTargetBits = QS_LANE_TARGET_BITS;

template <typename R>
static hipError_t sweep_u1_t(R *psi, int n, int S, int q, const double *tab_row, hipStream_t st)
{
    constexpr int VEC = kVec<R>;
    constexpr int U = 2;
    const uint64_t N = 1ull << n;
    // targets among the bits of a wave's 64 consecutive vectors (except complex<float> q = 0,
    // whose pair is one vector): lanes exchange partners instead of striding in memory
    const int lb = q - (VEC == 2 ? 1 : 0);
    if (lb >= 0 && lb < kLaneTargetBits && N / VEC >= 256 * U) {
        int log_items = n - (VEC == 2 ? 1 : 0);
        uint64_t total = (uint64_t)S << log_items;
        hipLaunchKernelGGL((k_u1_lane<R, U>), dim3(blocks_for(total, 256 * U)), dim3(256), 0, st, psi, n, lb,
                           tab_row, log_items, total);
    } else if (q >= (VEC == 2 ? 1 : 0) && (N / 2) / VEC >= 256 * U) {
        int log_items = n - 1 - (VEC == 2 ? 1 : 0);
        uint64_t total = (uint64_t)S << log_items;
        hipLaunchKernelGGL((k_u1<R, 0, U>), dim3(blocks_for(total, 256 * U)), dim3(256), 0, st, psi,
                           n, q, tab_row, log_items, total);
    } else if (VEC == 2 && q == 0 && (N / 2) >= 256 * U) {
        int log_items = n - 1;
        uint64_t total = (uint64_t)S << log_items;
        hipLaunchKernelGGL((k_u1<R, 1, U>), dim3(blocks_for(total, 256 * U)), dim3(256), 0, st, psi,
                           n, q, tab_row, log_items, total);
    } else {
        uint64_t total = (uint64_t)S << (n - 1);
        hipLaunchKernelGGL(k_u1_small<R>, dim3(blocks_for(total, 256)), dim3(256), 0, st, psi, n,
                           q, tab_row, total);
    }
    return hipGetLastError();
}

hipError_t launch_sweep_u1(void *psi, qs_dtype dt, int n, int S, int q, const double *tab_row,
                           hipStream_t st)
{
    TimedLaunch tl("sweep_u1", 2.0 * (double)((uint64_t)S << n) * amp_bytes(dt), st);
    if (dt == QS_C64) return sweep_u1_t((float *)psi, n, S, q, tab_row, st);
    return sweep_u1_t((double *)psi, n, S, q, tab_row, st);
}

template <typename R, int KIND>
static hipError_t sweep_2q_t(R *psi, int n, int S, int qa, int qb, const double *tab_row,
                             const double *m32_host, hipStream_t st)
{
    M32 m32{};
    if (m32_host)
        for (int k = 0; k < 32; ++k) m32.v[k] = m32_host[k];
    constexpr int VEC = kVec<R>;
    const int lo = qa < qb ? qa : qb;
    if (VEC == 2 && lo >= 1 && n >= 3) {
        int log_items = n - 3;
        uint64_t total = (uint64_t)S << log_items;
        hipLaunchKernelGGL((k_2q<R, KIND, 2>), dim3(blocks_for(total, 256)), dim3(256), 0, st, psi,
                           n, qa, qb, tab_row, m32, log_items, total);
    } else {
        int log_items = n - 2;
        uint64_t total = (uint64_t)S << log_items;
        hipLaunchKernelGGL((k_2q<R, KIND, 1>), dim3(blocks_for(total, 256)), dim3(256), 0, st, psi,
                           n, qa, qb, tab_row, m32, log_items, total);
    }
    return hipGetLastError();
}

hipError_t launch_sweep_cp(void *psi, qs_dtype dt, int n, int S, int qa, int qb,
                           const double *tab_row, hipStream_t st)
{
    TimedLaunch tl("sweep_cp", 2.0 * (double)((uint64_t)S << n) / 4 * amp_bytes(dt), st);
    if (dt == QS_C64) return sweep_2q_t<float, 0>((float *)psi, n, S, qa, qb, tab_row, nullptr, st);
    return sweep_2q_t<double, 0>((double *)psi, n, S, qa, qb, tab_row, nullptr, st);
}

hipError_t launch_sweep_perm(void *psi, qs_dtype dt, int n, int S, int kind, int qa, int qb,
                             hipStream_t st)
{
    TimedLaunch tl("sweep_swap", 2.0 * (double)((uint64_t)S << n) / 2 * amp_bytes(dt), st);
    if (kind == QS_G_SWAP) {
        if (dt == QS_C64) return sweep_2q_t<float, 1>((float *)psi, n, S, qa, qb, nullptr, nullptr, st);
        return sweep_2q_t<double, 1>((double *)psi, n, S, qa, qb, nullptr, nullptr, st);
    }
    if (dt == QS_C64) return sweep_2q_t<float, 2>((float *)psi, n, S, qa, qb, nullptr, nullptr, st);
    return sweep_2q_t<double, 2>((double *)psi, n, S, qa, qb, nullptr, nullptr, st);
}

// ---------------------------------------------------------------------------------------
// Dense 16x16 update on four index bits (the superoperator of a two-qubit Kraus set on
// vec(rho), eq. 3): for every index with those bits clear, the 16 entries whose local index
// l = sum_k bit(k of l) << bits[k] are replaced by M times them.  M is 256 complex FP64 values
// in device memory, row-major, read with uniform loads.
// ---------------------------------------------------------------------------------------
struct Bits4 {
    int b[4];        // the four index bits, local bit k -> index bit b[k]
    int sorted[4];   // the same, ascending (for inserting the zero bits)
};

template <typename R>
__global__ void __launch_bounds__(256) k_4q(R *psi, Bits4 bits, const double *__restrict__ m, uint64_t total)
{
    for (uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t base = g;
#pragma unroll
        for (int k = 0; k < 4; ++k) base = ins0(base, bits.sorted[k]);
        uint64_t idx[16];
        cx<R> x[16];
#pragma unroll
        for (int l = 0; l < 16; ++l) {
            uint64_t i = base;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if ((l >> k) & 1) i |= 1ull << bits.b[k];
            idx[l] = i;
            x[l] = sload(psi, i);
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            cx<R> y = {(R)0, (R)0};
#pragma unroll
            for (int c = 0; c < 16; ++c) {
                const cx<R> mrc = {(R)m[2 * (16 * r + c)], (R)m[2 * (16 * r + c) + 1]};
                y = cfma(mrc, x[c], y);
            }
            sstore(psi, idx[r], y);
        }
    }
}

hipError_t launch_sweep_4q(void *psi, qs_dtype dt, int nbits, const int bits[4], const double *m_dev,
                           hipStream_t st)
{
    Bits4 b{};
    for (int k = 0; k < 4; ++k) b.b[k] = b.sorted[k] = bits[k];
    std::sort(b.sorted, b.sorted + 4);
    const uint64_t total = 1ull << (nbits - 4);
    TimedLaunch tl("sweep_4q", 2.0 * (double)(1ull << nbits) * amp_bytes(dt), st);
    if (dt == QS_C64)
        hipLaunchKernelGGL(k_4q<float>, dim3(blocks_for(total, 256)), dim3(256), 0, st, (float *)psi, b, m_dev,
                           total);
    else
        hipLaunchKernelGGL(k_4q<double>, dim3(blocks_for(total, 256)), dim3(256), 0, st, (double *)psi, b, m_dev,
                           total);
    return hipGetLastError();
}

// The lane form of the dense two-qubit sweep when the lower qubit is among a wave's lane bits
// and the upper one above the wave's vectors; false when it does not apply.
template <typename R>
static bool sweep_2q_lane(R *psi, int n, int S, int qa, int qb, const double *m32_host, hipStream_t st)
{
    constexpr int VEC = kVec<R>;
    constexpr int vbits = VEC == 2 ? 1 : 0;
    const int lo = qa < qb ? qa : qb, hi = qa < qb ? qb : qa;
    const int lb = lo - vbits, hb = hi - vbits;
    if (lb < 0 || lb >= kLaneTargetBits || hb < 6 || n - vbits - 1 < 8) return false;
    // the kernel takes the lower qubit as the low local bit: when qa is the upper one, swap the
    // two bits of both local indices (local index bit(qa) + 2 bit(qb))
    M32 m{};
    auto sw = [&](int l) { return qa == lo ? l : ((l & 1) << 1) | (l >> 1); };
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            m.v[2 * (4 * sw(r) + sw(c))] = m32_host[2 * (4 * r + c)];
            m.v[2 * (4 * sw(r) + sw(c)) + 1] = m32_host[2 * (4 * r + c) + 1];
        }
    const int log_items = n - vbits - 1;
    const uint64_t total = (uint64_t)S << log_items;
    hipLaunchKernelGGL(k_2q_lane<R>, dim3(blocks_for(total, 256)), dim3(256), 0, st, psi, n, lb, hb, m,
                       log_items, total);
    return true;
}

hipError_t launch_sweep_2q(void *psi, qs_dtype dt, int n, int S, int qa, int qb,
                           const double *m32, hipStream_t st)
{
    TimedLaunch tl("sweep_2q", 2.0 * (double)((uint64_t)S << n) * amp_bytes(dt), st);
    if (dt == QS_C64 ? sweep_2q_lane((float *)psi, n, S, qa, qb, m32, st)
                     : sweep_2q_lane((double *)psi, n, S, qa, qb, m32, st))
        return hipGetLastError();
    if (dt == QS_C64) return sweep_2q_t<float, 3>((float *)psi, n, S, qa, qb, nullptr, m32, st);
    return sweep_2q_t<double, 3>((double *)psi, n, S, qa, qb, nullptr, m32, st);
}

hipError_t launch_flip(void *psi, qs_dtype dt, int n, int S, uint64_t mask, uint64_t value,
                       hipStream_t st)
{
    mask &= (n >= 64) ? ~0ull : ((1ull << n) - 1);
    int free_bits = n - __builtin_popcountll(mask);
    uint64_t total = (uint64_t)S << free_bits;
    TimedLaunch tl("flip", 2.0 * (double)total * amp_bytes(dt), st);
    if (dt == QS_C64)
        hipLaunchKernelGGL(k_flip<float>, dim3(blocks_for(total, 256)), dim3(256), 0, st,
                           (float *)psi, n, mask, value, free_bits, total);
    else
        hipLaunchKernelGGL(k_flip<double>, dim3(blocks_for(total, 256)), dim3(256), 0, st,
                           (double *)psi, n, mask, value, free_bits, total);
    return hipGetLastError();
}

hipError_t launch_scale_pattern(void *psi, qs_dtype dt, int n, int S, uint64_t mask, uint64_t value,
                                double fre, double fim, hipStream_t st)
{
    const int free_bits = n - __builtin_popcountll(mask);
    const uint64_t total = (uint64_t)S << free_bits;
    TimedLaunch tl("flip", 2.0 * (double)total * amp_bytes(dt), st);
    if (dt == QS_C64)
        hipLaunchKernelGGL(k_scale_pattern<float>, dim3(blocks_for(total, 256)), dim3(256), 0, st,
                           (float *)psi, n, mask, value, free_bits, total, fre, fim);
    else
        hipLaunchKernelGGL(k_scale_pattern<double>, dim3(blocks_for(total, 256)), dim3(256), 0, st,
                           (double *)psi, n, mask, value, free_bits, total, fre, fim);
    return hipGetLastError();
}

size_t reduce_partials_doubles(int n, int S)
{
    size_t a = ((size_t)S << red_log_blocks(n)) * 3;
    int ld = red_log_blocks(2 * n) ;
    size_t b = ((size_t)1 << ld) * 4;
    return a > b ? a : b;
}

hipError_t launch_overlap_final(const void *psi, qs_dtype dt, int n, int S, int log_blocks, int64_t marked,
                                const double *partials, double *out, hipStream_t st, const RunParams *dyn)
{
    TimedLaunch tl("reduce", (double)((uint64_t)S << log_blocks) * 3 * sizeof(double), st);
    if (dt == QS_C64)
        hipLaunchKernelGGL(k_overlap_final<float>, dim3(S), dim3(kRedThreads), 0, st, (const float *)psi, n,
                           log_blocks, marked, partials, out, dyn);
    else
        hipLaunchKernelGGL(k_overlap_final<double>, dim3(S), dim3(kRedThreads), 0, st, (const double *)psi, n,
                           log_blocks, marked, partials, out, dyn);
    return hipGetLastError();
}

hipError_t launch_overlaps(const void *ref_psi, int ref_slot, const void *psi, qs_dtype dt, int n,
                           int S, int64_t marked, double *partials, double *out, hipStream_t st,
                           const RunParams *dyn)
{
    int lb = red_log_blocks(n);
    unsigned nblk = (unsigned)((uint64_t)S << lb);
    // algorithmic bytes: every state once and the reference once
    TimedLaunch tl("reduce", (double)((uint64_t)(S + 1) << n) * amp_bytes(dt), st);
    if (dt == QS_C64) {
        const float *ref = (const float *)ref_psi + ((uint64_t)ref_slot << (n + 1));
        hipLaunchKernelGGL(k_overlap_partial<float>, dim3(nblk), dim3(kRedThreads), 0, st, ref,
                           (const float *)psi, n, lb, partials);
        hipLaunchKernelGGL(k_overlap_final<float>, dim3(S), dim3(kRedThreads), 0, st,
                           (const float *)psi, n, lb, marked, partials, out, dyn);
    } else {
        const double *ref = (const double *)ref_psi + ((uint64_t)ref_slot << (n + 1));
        hipLaunchKernelGGL(k_overlap_partial<double>, dim3(nblk), dim3(kRedThreads), 0, st, ref,
                           (const double *)psi, n, lb, partials);
        hipLaunchKernelGGL(k_overlap_final<double>, dim3(S), dim3(kRedThreads), 0, st,
                           (const double *)psi, n, lb, marked, partials, out, dyn);
    }
    return hipGetLastError();
}

hipError_t launch_dm_expect(const void *rho, const void *psi, qs_dtype dt, int n,
                            double *partials, double *out, hipStream_t st)
{
    int lb = red_log_blocks(2 * n);
    TimedLaunch tl("reduce", (double)((uint64_t)1 << (2 * n)) * amp_bytes(dt), st);
    if (dt == QS_C64)
        hipLaunchKernelGGL(k_dm_expect_partial<float>, dim3(1u << lb), dim3(kRedThreads), 0, st,
                           (const float *)rho, (const float *)psi, n, lb, partials);
    else
        hipLaunchKernelGGL(k_dm_expect_partial<double>, dim3(1u << lb), dim3(kRedThreads), 0, st,
                           (const double *)rho, (const double *)psi, n, lb, partials);
    hipLaunchKernelGGL(k_sum4_final, dim3(1), dim3(kRedThreads), 0, st, partials, 1 << lb, out);
    return hipGetLastError();
}

// dst[sigma(i)] = src[i] over the n-bit indices i, sigma moving bit q of i to bit perm[q] (one
// state vector; sigma must be a permutation of 0..n-1).
struct BitPerm {
    int8_t p[40];
};

template <typename R>
__global__ void k_permute_bits(R *dst, const R *src, int n, BitPerm bp, uint64_t total)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t j = 0;
        for (int q = 0; q < n; ++q)
            if ((i >> q) & 1ull) j |= 1ull << bp.p[q];
        dst[2 * j] = src[2 * i];
        dst[2 * j + 1] = src[2 * i + 1];
    }
}

hipError_t launch_permute_bits(void *dst, const void *src, qs_dtype dt, int n, const int32_t *perm,
                               hipStream_t st)
{
    if (n < 1 || n > 40) return hipErrorInvalidValue;
    BitPerm bp{};
    for (int q = 0; q < n; ++q) bp.p[q] = (int8_t)perm[q];
    const uint64_t total = 1ull << n;
    TimedLaunch tl("copy", 2.0 * (double)total * amp_bytes(dt), st);
    unsigned blocks = (unsigned)std::min<uint64_t>(blocks_for(total, 256), 256u * 64u);
    if (dt == QS_C64)
        hipLaunchKernelGGL(k_permute_bits<float>, dim3(blocks), dim3(256), 0, st, (float *)dst,
                           (const float *)src, n, bp, total);
    else
        hipLaunchKernelGGL(k_permute_bits<double>, dim3(blocks), dim3(256), 0, st, (double *)dst,
                           (const double *)src, n, bp, total);
    return hipGetLastError();
}

hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t st)
{
    uint64_t n16 = bytes / 16;
    TimedLaunch tl("copy", 2.0 * (double)bytes, st);
    unsigned blocks = (unsigned)std::min<uint64_t>(blocks_for(n16, 256), 256u * 64u);
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, st, (float4 *)dst, (const float4 *)src, n16);
    return hipGetLastError();
}

}  // namespace qs
