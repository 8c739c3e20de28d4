// Fused pass kernel: a run of gates whose non-diagonal targets lie in one set of K "tile"
// qubits is applied to every tile of 2^K amplitudes in a single read and write of HBM.
//
// Layout: tile-local index bit j is physical bit q_pos[j]; the other n - K bits number the
// tiles (one workgroup per tile and slot).  Each thread keeps 2^RB amplitudes in registers.
// A round names the RB tile-local bits held in registers; a one-qubit gate on one of them
// updates register pairs (Section 2's amplitude-pair update), a two-qubit gate register
// quadruples.  Between rounds the tile is re-distributed through LDS.  Controlled phases and
// sign flips are diagonal: a controlled phase is folded into the neighbouring one-qubit gate
// on one of its qubits as a phase on that gate's |1> input or output, conditioned on the other
// qubit, which is a tile-constant, thread-constant or register bit here.
#include "internal.h"

namespace qs {

template <typename R>
struct cxf {
    R re, im;
};

template <typename R>
__device__ __forceinline__ cxf<R> mul(cxf<R> a, cxf<R> b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

template <typename R>
__device__ __forceinline__ cxf<R> fma_c(cxf<R> a, cxf<R> b, cxf<R> c)
{
    return {a.re * b.re - a.im * b.im + c.re, a.re * b.im + a.im * b.re + c.im};
}

template <typename R>
__device__ __forceinline__ cxf<R> ld_tab(const double *t)
{
    return {(R)t[0], (R)t[1]};
}

// LDS slot of tile-local index l: the low five bits are xor-ed with a fold of the higher bits,
// a bijection that spreads strided accesses over the banks.
__device__ __forceinline__ uint32_t swz(uint32_t l)
{
    return l ^ (((l >> 5) ^ (l >> 10)) & 31u);
}

// Deposit the low bits of x into the set bits of mask (lowest first).
__device__ __forceinline__ uint32_t deposit32(uint32_t x, uint32_t mask, int K)
{
    uint32_t out = 0;
    int b = 0;
    for (int j = 0; j < K; ++j) {
        if (mask & (1u << j)) {
            out |= ((x >> b) & 1u) << j;
            ++b;
        }
    }
    return out;
}

template <int RB>
__device__ __forceinline__ void reg_offsets(uint32_t reg_mask, int K, uint32_t (&roff)[1 << RB])
{
    uint32_t pos[RB];
    int b = 0;
    for (int j = 0; j < K && b < RB; ++j)
        if (reg_mask & (1u << j)) pos[b++] = 1u << j;
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r) {
        uint32_t o = 0;
#pragma unroll
        for (int k = 0; k < RB; ++k)
            if (r & (1 << k)) o |= pos[k];
        roff[r] = o;
    }
}

template <typename R, int RB>
struct PhaseSet {
    cxf<R> w;          // tile/thread-constant factor
    cxf<R> bit[RB];    // factor per register bit (applied when that bit of the pair index is 1)
    bool any;
    bool reg;
};

template <typename R, int RB>
__device__ __forceinline__ void gather_phases(PhaseSet<R, RB> &ps, const PhaseRef *prefs, int b,
                                              int e, const double *tab, int S, int slot,
                                              uint64_t outer, uint32_t lthr)
{
    ps.w = {(R)1, (R)0};
#pragma unroll
    for (int k = 0; k < RB; ++k) ps.bit[k] = {(R)1, (R)0};
    ps.any = e > b;
    ps.reg = false;
    for (int k = b; k < e; ++k) {
        const PhaseRef pr = prefs[k];
        cxf<R> ph = ld_tab<R>(tab + ((uint64_t)pr.gate * S + slot) * 8);
        if (pr.cls == PH_OUTER) {
            if ((outer >> pr.bit) & 1ull) ps.w = mul(ps.w, ph);
        } else if (pr.cls == PH_THREAD) {
            cxf<R> t = mul(ps.w, ph);
            bool on = (lthr >> pr.bit) & 1u;
            ps.w.re = on ? t.re : ps.w.re;
            ps.w.im = on ? t.im : ps.w.im;
        } else {
            ps.reg = true;
#pragma unroll
            for (int q = 0; q < RB; ++q)
                if (pr.bit == q) ps.bit[q] = mul(ps.bit[q], ph);
        }
    }
}

template <typename R, int RB, int P>
__device__ __forceinline__ cxf<R> pair_phase(const PhaseSet<R, RB> &ps, int r)
{
    cxf<R> w = ps.w;
    if (ps.reg) {
#pragma unroll
        for (int q = 0; q < RB; ++q)
            if (q != P && ((r >> q) & 1)) w = mul(w, ps.bit[q]);
    }
    return w;
}

template <typename R, int RB, int P>
__device__ __forceinline__ void apply_u1(cxf<R> (&a)[1 << RB], const cxf<R> (&m)[4],
                                         const PhaseSet<R, RB> &pre, const PhaseSet<R, RB> &post)
{
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r) {
        if (r & (1 << P)) continue;
        const int r1 = r | (1 << P);
        cxf<R> x0 = a[r], x1 = a[r1];
        if (pre.any) x1 = mul(pair_phase<R, RB, P>(pre, r), x1);
        cxf<R> y0 = fma_c(m[1], x1, mul(m[0], x0));
        cxf<R> y1 = fma_c(m[3], x1, mul(m[2], x0));
        if (post.any) y1 = mul(pair_phase<R, RB, P>(post, r), y1);
        a[r] = y0;
        a[r1] = y1;
    }
}

template <typename R, int RB, int P0, int P1>
__device__ __forceinline__ void apply_u2(cxf<R> (&a)[1 << RB], const cxf<R> (&m)[16])
{
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r) {
        if ((r & (1 << P0)) || (r & (1 << P1))) continue;
        const int idx[4] = {r, r | (1 << P0), r | (1 << P1), r | (1 << P0) | (1 << P1)};
        cxf<R> x[4] = {a[idx[0]], a[idx[1]], a[idx[2]], a[idx[3]]};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            cxf<R> s = mul(m[4 * i], x[0]);
            s = fma_c(m[4 * i + 1], x[1], s);
            s = fma_c(m[4 * i + 2], x[2], s);
            s = fma_c(m[4 * i + 3], x[3], s);
            a[idx[i]] = s;
        }
    }
}

template <typename R, int RB>
__device__ __forceinline__ void dispatch_u1(int p, cxf<R> (&a)[1 << RB], const cxf<R> (&m)[4],
                                            const PhaseSet<R, RB> &pre, const PhaseSet<R, RB> &post)
{
    switch (p) {
    case 0: apply_u1<R, RB, 0>(a, m, pre, post); break;
    case 1: if constexpr (RB > 1) apply_u1<R, RB, 1 % RB>(a, m, pre, post); break;
    case 2: if constexpr (RB > 2) apply_u1<R, RB, 2 % RB>(a, m, pre, post); break;
    case 3: if constexpr (RB > 3) apply_u1<R, RB, 3 % RB>(a, m, pre, post); break;
    default: break;
    }
}

template <typename R, int RB>
__device__ __forceinline__ void dispatch_u2(int p0, int p1, cxf<R> (&a)[1 << RB], const cxf<R> (&m)[16])
{
    if constexpr (RB >= 2) {
#define QS_U2_CASE(A, B)                                                              \
    if (p0 == (A) && p1 == (B)) {                                                     \
        if constexpr ((A) < RB && (B) < RB && (A) != (B)) apply_u2<R, RB, (A) % RB, (B) % RB>(a, m); \
        return;                                                                       \
    }
        QS_U2_CASE(0, 1) QS_U2_CASE(1, 0) QS_U2_CASE(0, 2) QS_U2_CASE(2, 0)
        QS_U2_CASE(0, 3) QS_U2_CASE(3, 0) QS_U2_CASE(1, 2) QS_U2_CASE(2, 1)
        QS_U2_CASE(1, 3) QS_U2_CASE(3, 1) QS_U2_CASE(2, 3) QS_U2_CASE(3, 2)
#undef QS_U2_CASE
    }
}

template <typename R, int RB>
__global__ void __launch_bounds__(512) k_fused(R *psi, int n, int S, const PassDesc *pd,
                                               const RoundDesc *rounds, const OpDesc *ops,
                                               const PhaseRef *prefs, const double *tab,
                                               const qs_gate *gates)
{
    extern __shared__ __align__(16) unsigned char smem[];
    cxf<R> *lds = reinterpret_cast<cxf<R> *>(smem);
    constexpr int NR = 1 << RB;
    const int K = pd->K;
    const int TB = K - RB;
    const uint32_t kmask = (K >= 32) ? 0xffffffffu : ((1u << K) - 1u);
    const int tiles_log = n - K;
    const int slot = (int)(blockIdx.x >> tiles_log);
    const uint64_t tile = (uint64_t)blockIdx.x & ((1ull << tiles_log) - 1ull);
    const uint32_t tid = threadIdx.x;

    // Outer (tile-number) bits of the physical index.
    uint64_t outer = 0;
    {
        uint64_t m = pd->outer_mask, t = tile;
        while (m) {
            uint64_t low = m & (~m + 1ull);
            if (t & 1ull) outer |= low;
            t >>= 1;
            m ^= low;
        }
    }
    // Load layout: thread bits = tile-local bits 0..TB-1, register bits = TB..K-1.
    uint64_t gthr = outer;
    for (int j = 0; j < TB; ++j)
        if ((tid >> j) & 1u) gthr |= 1ull << pd->q_pos[j];
    uint64_t greg[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        uint64_t g = 0;
#pragma unroll
        for (int k = 0; k < RB; ++k)
            if (r & (1 << k)) g |= 1ull << pd->q_pos[TB + k];
        greg[r] = g;
    }
    R *base = psi + ((uint64_t)slot << (n + 1));
    cxf<R> a[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        uint64_t i = gthr | greg[r];
        if constexpr (sizeof(R) == 4) {
            float2 v = *reinterpret_cast<const float2 *>(base + 2 * i);
            a[r] = {v.x, v.y};
        } else {
            double2 v = *reinterpret_cast<const double2 *>(base + 2 * i);
            a[r] = {v.x, v.y};
        }
    }

    const uint32_t load_mask = (((1u << RB) - 1u) << TB) & kmask;
    uint32_t cur = load_mask;
    uint32_t roff[NR];
    reg_offsets<RB>(cur, K, roff);
    uint32_t lthr = deposit32(tid, ~cur & kmask, K);

    auto exchange = [&](uint32_t to) {
        __syncthreads();
#pragma unroll
        for (int r = 0; r < NR; ++r) lds[swz(lthr | roff[r])] = a[r];
        __syncthreads();
        cur = to;
        reg_offsets<RB>(cur, K, roff);
        lthr = deposit32(tid, ~cur & kmask, K);
#pragma unroll
        for (int r = 0; r < NR; ++r) a[r] = lds[swz(lthr | roff[r])];
    };

    for (int ri = pd->round_begin; ri < pd->round_end; ++ri) {
        const RoundDesc rd = rounds[ri];
        if (rd.reg_mask != cur) exchange(rd.reg_mask);
        for (int oi = rd.op_begin; oi < rd.op_end; ++oi) {
            const OpDesc op = ops[oi];
            if (op.type == OP_U1) {
                const double *t = tab + ((uint64_t)op.gate * S + slot) * 8;
                cxf<R> m[4] = {ld_tab<R>(t), ld_tab<R>(t + 2), ld_tab<R>(t + 4), ld_tab<R>(t + 6)};
                PhaseSet<R, RB> pre, post;
                gather_phases<R, RB>(pre, prefs, op.pre_begin, op.pre_end, tab, S, slot, outer, lthr);
                gather_phases<R, RB>(post, prefs, op.post_begin, op.post_end, tab, S, slot, outer, lthr);
                dispatch_u1<R, RB>(op.p0, a, m, pre, post);
            } else if (op.type == OP_U2) {
                const double *g = gates[op.gate].m;
                cxf<R> m[16];
#pragma unroll
                for (int k = 0; k < 16; ++k) m[k] = {(R)g[2 * k], (R)g[2 * k + 1]};
                dispatch_u2<R, RB>(op.p0, op.p1, a, m);
            } else {
                if ((outer & op.omask) != op.ovalue) continue;
                cxf<R> f = {(R)-1, (R)0};
                if (op.diag_kind == DIAG_PHASE)
                    f = ld_tab<R>(tab + ((uint64_t)op.gate * S + slot) * 8);
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    bool hit = ((lthr | roff[r]) & op.lmask) == op.lvalue;
                    cxf<R> y = mul(f, a[r]);
                    a[r].re = hit ? y.re : a[r].re;
                    a[r].im = hit ? y.im : a[r].im;
                }
            }
        }
    }
    if (cur != load_mask) exchange(load_mask);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        uint64_t i = gthr | greg[r];
        if constexpr (sizeof(R) == 4) {
            *reinterpret_cast<float2 *>(base + 2 * i) = make_float2(a[r].re, a[r].im);
        } else {
            *reinterpret_cast<double2 *>(base + 2 * i) = make_double2(a[r].re, a[r].im);
        }
    }
}

size_t fused_lds_bytes(qs_dtype dt, int K) { return (size_t(1) << K) * (dt == QS_C64 ? 8 : 16); }

template <typename R, int RB>
static hipError_t launch_t(R *psi, int n, int S, const PassDesc &h, const PassDesc *pd,
                           const RoundDesc *rounds, const OpDesc *ops, const PhaseRef *prefs,
                           const double *tab, const qs_gate *gates, size_t lds, hipStream_t st)
{
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void *)k_fused<R, RB>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    unsigned blocks = (unsigned)((uint64_t)S << (n - h.K));
    unsigned threads = 1u << (h.K - RB);
    hipLaunchKernelGGL((k_fused<R, RB>), dim3(blocks), dim3(threads), lds, st, psi, n, S, pd,
                       rounds, ops, prefs, tab, gates);
    return hipGetLastError();
}

hipError_t launch_fused_pass(void *psi, qs_dtype dt, int n, int S, const PassDesc *pass_host,
                             const PassDesc *pass_dev, const RoundDesc *rounds,
                             const OpDesc *ops, const PhaseRef *prefs, const double *tab,
                             const qs_gate *gates_dev, hipStream_t st)
{
    const PassDesc &h = *pass_host;
    size_t lds = fused_lds_bytes(dt, h.K);
    TimedLaunch tl("fused", 2.0 * (double)((uint64_t)S << n) * amp_bytes(dt), st);
    if (dt == QS_C64) {
        float *p = (float *)psi;
        switch (h.RB) {
        case 1: return launch_t<float, 1>(p, n, S, h, pass_dev, rounds, ops, prefs, tab, gates_dev, lds, st);
        case 2: return launch_t<float, 2>(p, n, S, h, pass_dev, rounds, ops, prefs, tab, gates_dev, lds, st);
        case 3: return launch_t<float, 3>(p, n, S, h, pass_dev, rounds, ops, prefs, tab, gates_dev, lds, st);
        case 4: return launch_t<float, 4>(p, n, S, h, pass_dev, rounds, ops, prefs, tab, gates_dev, lds, st);
        }
    } else {
        double *p = (double *)psi;
        switch (h.RB) {
        case 1: return launch_t<double, 1>(p, n, S, h, pass_dev, rounds, ops, prefs, tab, gates_dev, lds, st);
        case 2: return launch_t<double, 2>(p, n, S, h, pass_dev, rounds, ops, prefs, tab, gates_dev, lds, st);
        case 3: return launch_t<double, 3>(p, n, S, h, pass_dev, rounds, ops, prefs, tab, gates_dev, lds, st);
        case 4: return launch_t<double, 4>(p, n, S, h, pass_dev, rounds, ops, prefs, tab, gates_dev, lds, st);
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace qs
