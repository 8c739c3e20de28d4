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
#include <type_traits>

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

// Register-tile element: one complex amplitude as a two-lane vector, so that the compiler keeps
// it in an aligned register pair and moves it with one 64-bit move.
template <typename R>
using tv = R __attribute__((ext_vector_type(2)));
template <typename R>
__device__ __forceinline__ cxf<R> cx(tv<R> v) { return {v.x, v.y}; }
template <typename R>
__device__ __forceinline__ tv<R> tvec(cxf<R> c) { return tv<R>{c.re, c.im}; }

__device__ __forceinline__ uint32_t swz(uint32_t l)
{
    return lds_swizzle(l);
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

// Phase factors of one folded block for this thread: w (tile and thread constant) and one
// factor per register bit, applied to a pair when that bit of the pair index is 1.
template <typename R, int RB>
struct PhaseSet {
    cxf<R> w;
    cxf<R> bit[RB];
    bool any;
};

// grec: the block in global memory (uniform reads, held in scalar registers); lrec: the same
// block staged in LDS (per-thread table lookups); wout: this tile's products of the phases
// conditioned on tile-number bits (global memory, uniform reads).
// bits: whether the block has phases conditioned on register bits (else only w is used).
// uni: no factor of the block depends on a thread-id bit, so every entry of the thread tables
// equals their first (uniform reads instead of per-thread lookups).
template <typename R, int RB>
__device__ __forceinline__ void load_phases(PhaseSet<R, RB> &ps, const cxf<R> *__restrict__ grec,
                                            const cxf<R> *lrec, bool present, bool bits, bool uni, int job,
                                            const cxf<R> *wout, uint32_t tid)
{
    ps.any = present;
    if (!present) return;
    if (bits) {
#pragma unroll
        for (int k = 0; k < RB; ++k) ps.bit[k] = grec[k];
    }
    if (uni) ps.w = grec[4];
    else ps.w = mul(lrec[4 + (tid & 31u)], lrec[36 + ((tid >> 5) & 15u)]);
    if (job >= 0) ps.w = mul(ps.w, wout[job]);
}

// Phase of the pair at register index r: w, times the register-bit factors when BITS.
template <typename R, int RB, int P, bool BITS>
__device__ __forceinline__ cxf<R> pair_phase(const PhaseSet<R, RB> &ps, int r)
{
    cxf<R> w = ps.w;
    if constexpr (BITS) {
#pragma unroll
        for (int q = 0; q < RB; ++q)
            if (q != P && ((r >> q) & 1)) w = mul(w, ps.bit[q]);
    }
    return w;
}

// Register index of the k-th pair (bit P clear) and of the k-th quadruple (bits P0, P1 clear):
// compile-time integer arithmetic, so that after unrolling every register access is static.
template <int P>
__device__ constexpr int pair_base(int k)
{
    return ((k >> P) << (P + 1)) | (k & ((1 << P) - 1));
}

template <int P0, int P1>
__device__ constexpr int quad_base(int k)
{
    constexpr int lo = P0 < P1 ? P0 : P1, hi = P0 < P1 ? P1 : P0;
    return pair_base<hi>(pair_base<lo>(k));
}

// PRE: input phase kind (0 none, 1 one factor per thread, 2 with register-bit factors); POST:
// the folded output block (0 none, 1 one factor per thread, 2 with register-bit factors; with
// one factor it joins the |1> row of the matrix once per op instead of a product per pair).  ZIN: which input of every pair is known to be
// zero (0 neither; 1 the |1> input, 2 the |0> input) -- the target qubit has not been touched by
// any earlier gate of the run and still holds the basis bit 0 (1), so that half of the tile is
// exactly zero and its products are left out (the result is the same: a product with zero
// added to a value leaves the value).  They are uniform per op, so each combination is its own
// straight-line code behind a scalar branch, with no work for an absent block.
template <typename R, int RB, int P, int PRE, int POST, int ZIN>
__device__ __forceinline__ void apply_u1(tv<R> (&a)[1 << RB], const cxf<R> (&m0)[4],
                                         const PhaseSet<R, RB> &pre, const PhaseSet<R, RB> &post)
{
    cxf<R> m[4] = {m0[0], m0[1], m0[2], m0[3]};
    if constexpr (POST == 1) {
        m[2] = mul(post.w, m[2]);
        m[3] = mul(post.w, m[3]);
    }
#pragma unroll
    for (int k = 0; k < (1 << (RB - 1)); ++k) {
        const int r = pair_base<P>(k);
        const int r1 = r | (1 << P);
        cxf<R> x0 = cx<R>(a[r]), x1 = cx<R>(a[r1]);
        cxf<R> y0, y1;
        if constexpr (ZIN == 1) {
            y0 = mul(m[0], x0);
            y1 = mul(m[2], x0);
        } else {
            if constexpr (PRE > 0) x1 = mul(pair_phase<R, RB, P, PRE == 2>(pre, r), x1);
            if constexpr (ZIN == 2) {
                y0 = mul(m[1], x1);
                y1 = mul(m[3], x1);
            } else {
                y0 = fma_c(m[1], x1, mul(m[0], x0));
                y1 = fma_c(m[3], x1, mul(m[2], x0));
            }
        }
        if constexpr (POST == 2) y1 = mul(pair_phase<R, RB, P, true>(post, r), y1);
        a[r] = tvec(y0);
        a[r1] = tvec(y1);
    }
}

// The same update with a real matrix (m[k].im == 0): half the multiplications.  A one-factor
// output block makes the |1> row complex (m2 w, m3 w).
template <typename R, int RB, int P, int PRE, int POST, int ZIN>
__device__ __forceinline__ void apply_u1_real(tv<R> (&a)[1 << RB], const cxf<R> (&m)[4],
                                              const PhaseSet<R, RB> &pre, const PhaseSet<R, RB> &post)
{
    const R m0 = m[0].re, m1 = m[1].re, m2 = m[2].re, m3 = m[3].re;
    cxf<R> m2w, m3w;
    if constexpr (POST == 1) {
        m2w = {m2 * post.w.re, m2 * post.w.im};
        m3w = {m3 * post.w.re, m3 * post.w.im};
    }
#pragma unroll
    for (int k = 0; k < (1 << (RB - 1)); ++k) {
        const int r = pair_base<P>(k);
        const int r1 = r | (1 << P);
        cxf<R> x0 = cx<R>(a[r]), x1 = cx<R>(a[r1]);
        cxf<R> y0, y1;
        if constexpr (ZIN == 1) {
            y0 = {m0 * x0.re, m0 * x0.im};
            if constexpr (POST == 1) y1 = mul(m2w, x0);
            else y1 = {m2 * x0.re, m2 * x0.im};
        } else {
            if constexpr (PRE > 0) x1 = mul(pair_phase<R, RB, P, PRE == 2>(pre, r), x1);
            if constexpr (ZIN == 2) {
                y0 = {m1 * x1.re, m1 * x1.im};
                if constexpr (POST == 1) y1 = mul(m3w, x1);
                else y1 = {m3 * x1.re, m3 * x1.im};
            } else {
                y0 = {m0 * x0.re + m1 * x1.re, m0 * x0.im + m1 * x1.im};
                if constexpr (POST == 1) y1 = fma_c(m3w, x1, mul(m2w, x0));
                else y1 = {m2 * x0.re + m3 * x1.re, m2 * x0.im + m3 * x1.im};
            }
        }
        if constexpr (POST == 2) y1 = mul(pair_phase<R, RB, P, true>(post, r), y1);
        a[r] = tvec(y0);
        a[r1] = tvec(y1);
    }
}

// A one-qubit update on a target that still holds its basis bit, with a real matrix and one
// uniform output factor: one input of every pair is exactly zero (which one is the basis bit),
// so their sum is the other; the |0> output is A times it (A real), the |1> output B times it.
template <typename R, int RB, int P>
__device__ __forceinline__ void apply_u1_untouched(tv<R> (&a)[1 << RB], R A, cxf<R> B)
{
#pragma unroll
    for (int k = 0; k < (1 << (RB - 1)); ++k) {
        const int r = pair_base<P>(k);
        const int r1 = r | (1 << P);
        const cxf<R> x = {a[r].x + a[r1].x, a[r].y + a[r1].y};
        a[r] = tv<R>{A * x.re, A * x.im};
        a[r1] = tvec(mul(B, x));
    }
}

// REAL: the 4 x 4 matrix is real (a permutation, or the superoperator of a real Kraus set on
// vec(rho)): two multiply-adds per product instead of four.
template <typename R, int RB, int P0, int P1, bool REAL>
__device__ __forceinline__ void apply_u2(tv<R> (&a)[1 << RB], const cxf<R> (&m)[16])
{
#pragma unroll
    for (int k = 0; k < (1 << (RB - 2)); ++k) {
        const int r0 = quad_base<P0, P1>(k);
        const int r1 = r0 | (1 << P0), r2 = r0 | (1 << P1), r3 = r0 | (1 << P0) | (1 << P1);
        const cxf<R> x0 = cx<R>(a[r0]), x1 = cx<R>(a[r1]), x2 = cx<R>(a[r2]), x3 = cx<R>(a[r3]);
        cxf<R> y[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if constexpr (REAL) {
                const R c0 = m[4 * i].re, c1 = m[4 * i + 1].re, c2 = m[4 * i + 2].re, c3 = m[4 * i + 3].re;
                y[i] = {c0 * x0.re + c1 * x1.re + c2 * x2.re + c3 * x3.re,
                        c0 * x0.im + c1 * x1.im + c2 * x2.im + c3 * x3.im};
            } else {
                cxf<R> s = mul(m[4 * i], x0);
                s = fma_c(m[4 * i + 1], x1, s);
                s = fma_c(m[4 * i + 2], x2, s);
                s = fma_c(m[4 * i + 3], x3, s);
                y[i] = s;
            }
        }
        a[r0] = tvec(y[0]);
        a[r1] = tvec(y[1]);
        a[r2] = tvec(y[2]);
        a[r3] = tvec(y[3]);
    }
}

// Dispatch on the target register bit.  There is no pass-through branch (the last position
// is the fall-back): every path rewrites the register tile, which lets the register allocator
// keep the tile in the same registers across ops instead of copying it at each merge.
template <typename R, int RB, int PRE, int POST, int ZIN>
__device__ __forceinline__ void dispatch_u1_pp(int p, bool real, tv<R> (&a)[1 << RB], const cxf<R> (&m)[4],
                                               const PhaseSet<R, RB> &pre, const PhaseSet<R, RB> &post)
{
    if (real) {
        if (RB > 1 && p == 0) apply_u1_real<R, RB, 0, PRE, POST, ZIN>(a, m, pre, post);
        else if (RB > 2 && p == 1) apply_u1_real<R, RB, 1 % RB, PRE, POST, ZIN>(a, m, pre, post);
        else if (RB > 3 && p == 2) apply_u1_real<R, RB, 2 % RB, PRE, POST, ZIN>(a, m, pre, post);
        else apply_u1_real<R, RB, RB - 1, PRE, POST, ZIN>(a, m, pre, post);
        return;
    }
    if (RB > 1 && p == 0) apply_u1<R, RB, 0, PRE, POST, ZIN>(a, m, pre, post);
    else if (RB > 2 && p == 1) apply_u1<R, RB, 1 % RB, PRE, POST, ZIN>(a, m, pre, post);
    else if (RB > 3 && p == 2) apply_u1<R, RB, 2 % RB, PRE, POST, ZIN>(a, m, pre, post);
    else apply_u1<R, RB, RB - 1, PRE, POST, ZIN>(a, m, pre, post);
}

// zin: 0 general, 1 the |1> inputs are zero (no input phase to apply), 2 the |0> inputs are zero.
// postkind: 0 no output block, 1 one factor per thread, 2 with register-bit factors.
template <typename R, int RB, int PRE, int ZIN>
__device__ __forceinline__ void dispatch_u1_post(int p, bool real, int postkind, tv<R> (&a)[1 << RB],
                                                 const cxf<R> (&m)[4], const PhaseSet<R, RB> &pre,
                                                 const PhaseSet<R, RB> &post)
{
    if (postkind == 2) dispatch_u1_pp<R, RB, PRE, 2, ZIN>(p, real, a, m, pre, post);
    else if (postkind == 1) dispatch_u1_pp<R, RB, PRE, 1, ZIN>(p, real, a, m, pre, post);
    else dispatch_u1_pp<R, RB, PRE, 0, ZIN>(p, real, a, m, pre, post);
}

template <typename R, int RB>
__device__ __forceinline__ void dispatch_u1(int p, bool real, int prekind, int zin, int postkind,
                                            tv<R> (&a)[1 << RB], const cxf<R> (&m)[4],
                                            const PhaseSet<R, RB> &pre, const PhaseSet<R, RB> &post)
{
    if (zin == 1) {
        dispatch_u1_post<R, RB, 0, 1>(p, real, postkind, a, m, pre, post);
    } else if (zin == 2) {
        if (prekind == 2) dispatch_u1_post<R, RB, 2, 2>(p, real, postkind, a, m, pre, post);
        else if (prekind == 1) dispatch_u1_post<R, RB, 1, 2>(p, real, postkind, a, m, pre, post);
        else dispatch_u1_post<R, RB, 0, 2>(p, real, postkind, a, m, pre, post);
    } else if (prekind == 2) {
        dispatch_u1_post<R, RB, 2, 0>(p, real, postkind, a, m, pre, post);
    } else if (prekind == 1) {
        dispatch_u1_post<R, RB, 1, 0>(p, real, postkind, a, m, pre, post);
    } else {
        dispatch_u1_post<R, RB, 0, 0>(p, real, postkind, a, m, pre, post);
    }
}

template <typename R, int RB, bool REAL>
__device__ __forceinline__ void dispatch_u2_t(int p0, int p1, tv<R> (&a)[1 << RB], const cxf<R> (&m)[16])
{
    if constexpr (RB >= 2) {
        switch (p0 * 4 + p1) {
#define QS_U2_CASE(A, B) \
    case (A) * 4 + (B): if constexpr ((A) < RB && (B) < RB) apply_u2<R, RB, (A) % RB, (B) % RB, REAL>(a, m); break;
        QS_U2_CASE(0, 1) QS_U2_CASE(1, 0) QS_U2_CASE(0, 2) QS_U2_CASE(2, 0)
        QS_U2_CASE(0, 3) QS_U2_CASE(3, 0) QS_U2_CASE(1, 2) QS_U2_CASE(2, 1)
        QS_U2_CASE(1, 3) QS_U2_CASE(3, 1) QS_U2_CASE(2, 3) QS_U2_CASE(3, 2)
#undef QS_U2_CASE
        default: break;
        }
    }
}

template <typename R, int RB>
__device__ __forceinline__ void dispatch_u2(int p0, int p1, bool real, tv<R> (&a)[1 << RB], const cxf<R> (&m)[16])
{
    if (real) dispatch_u2_t<R, RB, true>(p0, p1, a, m);
    else dispatch_u2_t<R, RB, false>(p0, p1, a, m);
}

// ---------------------------------------------------------------------------------------
// Dense 16 x 16 blocks on the FP32 matrix cores (rounds the planner marks with a block record).
// In a round the 16 registers of a thread are the 16 states of the round's four qubits (register
// index = block index) and the thread id numbers the columns.  A 16 x 16 x 4 product takes its
// K index from lane bits 4, 5 and a chunk index, so register bits 0, 1 are first exchanged with
// lane bits 4, 5 (one lane-half swap per register pair and component); then register
// g + 4c of lane group j holds block state j + 4c of column group g.  With the block as the real
// 32 x 32 matrix [[Re U, -Im U], [Im U, Re U]] acting on [Re x; Im x], eight products of four
// rows each give the real and imaginary output rows of one column group.  Output register i of
// lane group j holds row 4j + i; it is stored at register g + 4i, and after the exchange back
// the register index is j + 4i.  The operand table holds the block with its rows permuted by
// P(4j + i) = 4i + j, so that register j + 4i ends with output state j + 4i.
// ---------------------------------------------------------------------------------------
typedef float mf4 __attribute__((ext_vector_type(4)));

// (lo, hi): the same register pair of a lane half; exchange the upper 16 lanes of each 32 of lo
// with the lower 16 of hi (a transpose of register bit and lane bit 4).
__device__ __forceinline__ void lane_swap16(tv<float> &lo, tv<float> &hi)
{
    const auto x = __builtin_amdgcn_permlane16_swap(__float_as_uint(lo.x), __float_as_uint(hi.x), false, false);
    const auto y = __builtin_amdgcn_permlane16_swap(__float_as_uint(lo.y), __float_as_uint(hi.y), false, false);
    lo = tv<float>{__uint_as_float(x[0]), __uint_as_float(y[0])};
    hi = tv<float>{__uint_as_float(x[1]), __uint_as_float(y[1])};
}

// The same for lane bit 5 (upper 32 lanes of lo with the lower 32 of hi).
__device__ __forceinline__ void lane_swap32(tv<float> &lo, tv<float> &hi)
{
    const auto x = __builtin_amdgcn_permlane32_swap(__float_as_uint(lo.x), __float_as_uint(hi.x), false, false);
    const auto y = __builtin_amdgcn_permlane32_swap(__float_as_uint(lo.y), __float_as_uint(hi.y), false, false);
    lo = tv<float>{__uint_as_float(x[0]), __uint_as_float(y[0])};
    hi = tv<float>{__uint_as_float(x[1]), __uint_as_float(y[1])};
}

__device__ __forceinline__ void swap_reg01_lane45(tv<float> (&a)[16])
{
#pragma unroll
    for (int r = 0; r < 16; ++r)
        if (!(r & 1)) lane_swap16(a[r], a[r | 1]);
#pragma unroll
    for (int r = 0; r < 16; ++r)
        if (!(r & 2)) lane_swap32(a[r], a[r | 2]);
}

// y = U x for every column of the register tile (64 products); tab: this lane's 16 operand
// values, entry ob * 8 + c = row block ob (real, imaginary outputs) and K chunk c (rows 4c..4c+3
// of [Re x; Im x]).
__device__ __forceinline__ void block_apply(tv<float> (&a)[16], const float (&A)[16])
{
    swap_reg01_lane45(a);
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        mf4 re = {0.f, 0.f, 0.f, 0.f}, im = re;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            re = __builtin_amdgcn_mfma_f32_16x16x4f32(A[c], a[g + 4 * c].x, re, 0, 0, 0);
            im = __builtin_amdgcn_mfma_f32_16x16x4f32(A[8 + c], a[g + 4 * c].x, im, 0, 0, 0);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            re = __builtin_amdgcn_mfma_f32_16x16x4f32(A[4 + c], a[g + 4 * c].y, re, 0, 0, 0);
            im = __builtin_amdgcn_mfma_f32_16x16x4f32(A[12 + c], a[g + 4 * c].y, im, 0, 0, 0);
        }
        // column group g's inputs are consumed: its outputs take their registers
#pragma unroll
        for (int i = 0; i < 4; ++i) a[g + 4 * i] = tv<float>{re[i], im[i]};
    }
    swap_reg01_lane45(a);
}

// a[r] *= w for the registers whose bit P is set (a phase on the |1> state of register bit P).
template <typename R, int RB, int P>
__device__ __forceinline__ void phase_on_bit(tv<R> (&a)[1 << RB], cxf<R> w)
{
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r)
        if ((r >> P) & 1) a[r] = tvec(mul(w, cx<R>(a[r])));
}

template <typename R, int RB>
__device__ __forceinline__ void dispatch_phase_on_bit(int p, tv<R> (&a)[1 << RB], cxf<R> w)
{
    if (RB > 1 && p == 0) phase_on_bit<R, RB, 0>(a, w);
    else if (RB > 2 && p == 1) phase_on_bit<R, RB, 1 % RB>(a, w);
    else if (RB > 3 && p == 2) phase_on_bit<R, RB, 2 % RB>(a, w);
    else phase_on_bit<R, RB, RB - 1>(a, w);
}

// ---------------------------------------------------------------------------------------
// Per-slot records of one pass (one thread per op and slot; FP64 products rounded once).
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ double2 dmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ double2 dconj(double2 a) { return make_double2(a.x, -a.y); }

// a / |a| (1 for a == 0)
__device__ __forceinline__ double2 dunit(double2 a)
{
    const double h = hypot(a.x, a.y);
    return h > 0.0 ? make_double2(a.x / h, a.y / h) : make_double2(1.0, 0.0);
}

// Per (slot, block round, column): column `col` of the round's block U (the ops applied in order
// to the basis state col, in FP64: each op's phases conditioned on register bits on its |1> input,
// its 2 x 2 matrix, the same on its output), written into the operand table with rows permuted
// as block_apply expects.  The matrices and register-bit factors come from the slot's records,
// written by k_pass_prep before.
template <typename R>
__global__ void k_block_prep(int S, int round_begin, int n_rounds, int rec_size, ProgramDev prog,
                             cxf<R> *__restrict__ rec_all)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)S * n_rounds * 16) return;
    const int col = (int)(t & 15);
    const int rr = (int)((t >> 4) % n_rounds);
    const int slot = (int)((t >> 4) / n_rounds);
    const RoundDesc &rd = prog.rounds[round_begin + rr];
    if (rd.block_rec < 0) return;
    cxf<R> *rec = rec_all + (size_t)slot * rec_size;
    double2 v[16];
    for (int b = 0; b < 16; ++b) v[b] = make_double2(b == col ? 1.0 : 0.0, 0.0);
    auto ld = [&](int e) { return make_double2((double)rec[e].re, (double)rec[e].im); };
    auto bit_phases = [&](int block, int p) {
        if (block < 0) return;
        double2 f[4];
        for (int k = 0; k < 4; ++k) f[k] = ld(block + k);
        for (int b = 0; b < 16; ++b) {
            if (!((b >> p) & 1)) continue;
            double2 w = make_double2(1.0, 0.0);
            for (int k = 0; k < 4; ++k)
                if (k != p && ((b >> k) & 1)) w = dmul(w, f[k]);
            v[b] = dmul(w, v[b]);
        }
    };
    for (int oi = rd.op_begin; oi < rd.op_end; ++oi) {
        const OpDesc &op = prog.ops[oi];
        const int p = op.p0;
        bit_phases(op.pre_rec, p);
        const double2 m0 = ld(op.rec), m1 = ld(op.rec + 1), m2 = ld(op.rec + 2), m3 = ld(op.rec + 3);
        for (int b = 0; b < 16; ++b) {
            if ((b >> p) & 1) continue;
            const double2 x0 = v[b], x1 = v[b | (1 << p)];
            const double2 y0 = dmul(m0, x0), y0b = dmul(m1, x1), y1 = dmul(m2, x0), y1b = dmul(m3, x1);
            v[b] = make_double2(y0.x + y0b.x, y0.y + y0b.y);
            v[b | (1 << p)] = make_double2(y1.x + y1b.x, y1.y + y1b.y);
        }
        bit_phases(op.post_rec, p);
    }
    // U[g][col] = v[g] goes to row P(g) of the permuted block; real form entries
    // (r, c) -> lane (r % 16) + 16 (c % 4), entry (r / 16) * 8 + c / 4 of the lane's 16
    R *tab = reinterpret_cast<R *>(rec + rd.block_rec);
    auto put = [&](int r, int c, double x) { tab[((r & 15) + 16 * (c & 3)) * 16 + (r >> 4) * 8 + (c >> 2)] = (R)x; };
    for (int g = 0; g < 16; ++g) {
        const int r = ((g & 3) << 2) | (g >> 2);
        put(r, col, v[g].x);
        put(r, 16 + col, -v[g].y);
        put(16 + r, col, v[g].y);
        put(16 + r, 16 + col, v[g].x);
    }
}

// ---------------------------------------------------------------------------------------
// Phase chains (one thread per chain and slot, FP64).  Along a chain of one-qubit gates on
// one wire, each inner gate's matrix M (with the phase carried from the gate before it
// multiplied into its |1> column) is factored as M = p * diag(1, b) * Rm * diag(1, d) with
// unit p, b, d and Rm real.  Its row is rewritten as Rm in words 0, 2, 4, 6 and the input
// phase d in words 1, 3; b is carried to the next gate, p into the global phase, which the
// last gate of the chain takes along with the carried b (its row stays a complex matrix).
// The factors: p = phase(M00), d = phase(M01) / p, and b from the larger of the second row's
// entries, phase(M11) / (p d) or -phase(M10) / p; Rm is the real part of M with those phases
// divided out.  For a unitary M (M10 = -e^{it} conj(M01), M11 = e^{it} conj(M00)) the
// divided-out entries are real, so the factors reproduce M; a phase taken from a zero or
// rounding-sized entry only affects entries of that size.  (phase(0) = 1.)
// ---------------------------------------------------------------------------------------
__global__ void k_phase_chains(double *tab, int S, const int32_t *chain_gates, const int32_t *chain_off,
                               int n_chains)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_chains * S) return;
    const int c = (int)(i / S), s = (int)(i % S);
    const int kb = chain_off[c], ke = chain_off[c + 1];
    double2 carry = make_double2(1.0, 0.0), glob = make_double2(1.0, 0.0);
    for (int k = kb; k < ke; ++k) {
        double *t = tab + ((int64_t)chain_gates[k] * S + s) * 8;
        const double2 m00 = make_double2(t[0], t[1]), m10 = make_double2(t[4], t[5]);
        const double2 m01 = dmul(make_double2(t[2], t[3]), carry);
        const double2 m11 = dmul(make_double2(t[6], t[7]), carry);
        if (k == ke - 1) {
            const double2 o[4] = {dmul(glob, m00), dmul(glob, m01), dmul(glob, m10), dmul(glob, m11)};
            for (int j = 0; j < 4; ++j) {
                t[2 * j] = o[j].x;
                t[2 * j + 1] = o[j].y;
            }
            break;
        }
        const double2 p = dunit(m00);
        const double2 d = dmul(dunit(m01), dconj(p));
        const double2 b = hypot(m11.x, m11.y) >= hypot(m10.x, m10.y)
                              ? dmul(dunit(m11), dconj(dmul(p, d)))
                              : dmul(make_double2(-1.0, 0.0), dmul(dunit(m10), dconj(p)));
        const double2 pb = dmul(p, b), pd = dmul(p, d);
        t[0] = dmul(m00, dconj(p)).x;
        t[2] = dmul(m01, dconj(pd)).x;
        t[4] = dmul(m10, dconj(pb)).x;
        t[6] = dmul(m11, dconj(dmul(pb, d))).x;
        t[1] = d.x;
        t[3] = d.y;
        t[5] = 0.0;
        t[7] = 0.0;
        carry = b;
        glob = dmul(glob, p);
    }
}

hipError_t launch_phase_chains(double *tab, int S, const int32_t *chain_gates, const int32_t *chain_off,
                               int n_chains, hipStream_t st)
{
    const int64_t tot = (int64_t)n_chains * S;
    if (tot <= 0) return hipSuccess;
    TimedLaunch tl("chains", (double)tot * 64.0, st);
    hipLaunchKernelGGL(k_phase_chains, dim3((unsigned)((tot + 127) / 128)), dim3(128), 0, st, tab, S,
                       chain_gates, chain_off, n_chains);
    return hipGetLastError();
}

// Per (slot, tile, outer job) of one pass: the product of the job's record entries whose
// tile-number bit is set in the tile's index, in the order the planner listed them.  Tiles are
// numbered as the fused kernel's blocks are (the walked tile-number bits, the others at their
// basis values), so a block finds its products at wtab + blockIdx * jobs.
// Also writes otab[tile]: the tile's tile-number bits of the physical index (the walked bits
// from the tile number, the others at the basis values), from the threads of slot 0, job 0.
template <typename R>
__global__ void k_pass_jobs(int S, int n_jobs, int tiles_log, uint64_t walk, uint64_t fixed_bits, int rec_size,
                            const OuterJob *__restrict__ jobs, const int32_t *__restrict__ obits,
                            const cxf<R> *__restrict__ rec_all, const RunParams *dyn, uint64_t classical,
                            cxf<R> *__restrict__ wtab, uint64_t *__restrict__ otab)
{
    // thread order (slot, job, tile): the threads of a wave share the job, so its descriptor,
    // condition bits and factors are uniform loads (n_jobs == 0: one row of threads for otab)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per_slot = (int64_t)(n_jobs > 0 ? n_jobs : 1) << tiles_log;
    if (i >= (int64_t)S * per_slot) return;
    const int slot = (int)(i / per_slot);
    const int64_t rem = i - (int64_t)slot * per_slot;
    const int j = (int)(rem >> tiles_log);
    uint64_t t = (uint64_t)rem & ((1ull << tiles_log) - 1ull);
    const uint64_t tile = t;
    if (dyn) fixed_bits = (uint64_t)dyn->init & classical;
    uint64_t outer = fixed_bits, m = walk;
    while (m) {
        const uint64_t low = m & (~m + 1ull);
        if (t & 1ull) outer |= low;
        t >>= 1;
        m ^= low;
    }
    if (slot == 0 && j == 0) otab[tile] = outer;
    if (n_jobs == 0) return;
    const OuterJob jb = jobs[j];
    const cxf<R> *rec = rec_all + (size_t)slot * rec_size;
    cxf<R> w = {(R)1, (R)0};
    for (int k = 0; k < jb.n; ++k)
        if ((outer >> obits[jb.bits_off + k]) & 1ull) w = mul(w, rec[jb.rec_off + k]);
    wtab[(((int64_t)slot << tiles_log) + (int64_t)tile) * n_jobs + j] = w;
}

template <typename R>
__global__ void k_pass_prep(int S, int op_begin, int n_ops, int rec_size, ProgramDev prog,
                            const double *tab, const qs_gate *gates, cxf<R> *rec_all, uint64_t basis,
                            const RunParams *dyn)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)n_ops * S) return;
    if (dyn) basis = dyn->init;
    const int slot = (int)(i / n_ops), ol = (int)(i % n_ops);
    const OpDesc op = prog.ops[op_begin + ol];
    cxf<R> *blk = rec_all + (size_t)slot * rec_size;
    cxf<R> *rec = blk + op.rec;
    auto tabc = [&](int g) {
        const double *t = tab + ((uint64_t)g * S + slot) * 8;
        return make_double2(t[0], t[1]);
    };
    auto put = [&](cxf<R> *dst, double2 v) { *dst = cxf<R>{(R)v.x, (R)v.y}; };
    if (op.type == OP_U1) {
        const double *t = tab + ((uint64_t)op.gate * S + slot) * 8;
        const bool chain = (op.flags & OPF_CHAIN) != 0;
        double2 uni = make_double2(1.0, 0.0);
        if (chain) {
            // phase-chain layout: the real matrix in the even words, the input phase in words
            // 1 and 3; the phase joins the folded input block, else record entry 4
            for (int k = 0; k < 4; ++k) put(rec + k, make_double2(t[2 * k], 0.0));
            uni = make_double2(t[1], t[3]);
            if (op.flags & OPF_UPHASE) put(rec + 4, uni);
        } else {
            for (int k = 0; k < 4; ++k) put(rec + k, make_double2(t[2 * k], t[2 * k + 1]));
        }
        for (int post = 0; post < 2; ++post) {
            int block = post ? op.post_rec : op.pre_rec;
            if (block < 0) continue;
            double2 preg[kMaxRegBits], ptid[9];
            double2 ubas = make_double2(1.0, 0.0);     // the block's basis-conditioned factors
            for (int k = 0; k < kMaxRegBits; ++k) preg[k] = make_double2(1.0, 0.0);
            for (int k = 0; k < 9; ++k) ptid[k] = make_double2(1.0, 0.0);
            for (int k = op.pref_begin; k < op.pref_end; ++k) {
                const PrepRef pr = prog.prefs[k];
                if (pr.post != post) continue;
                double2 ph = tabc(pr.gate);
                if (pr.kind == PR_REG) preg[pr.bit] = dmul(preg[pr.bit], ph);
                else if (pr.kind == PR_THREAD) ptid[pr.bit] = dmul(ptid[pr.bit], ph);
                else if (pr.kind == PR_BASIS) {
                    if ((basis >> pr.bit) & 1ull) ubas = dmul(ubas, ph);
                } else put(blk + pr.slot_entry, ph);
            }
            cxf<R> *b = blk + block;
            for (int k = 0; k < 4; ++k) put(b + k, k < kMaxRegBits ? preg[k] : make_double2(1.0, 0.0));
            for (int x = 0; x < 32; ++x) {
                double2 w = dmul(ubas, post ? make_double2(1.0, 0.0) : uni);
                for (int k = 0; k < 5; ++k)
                    if ((x >> k) & 1) w = dmul(w, ptid[k]);
                put(b + 4 + x, w);
            }
            for (int y = 0; y < 16; ++y) {
                double2 w = make_double2(1.0, 0.0);
                for (int k = 0; k < 4; ++k)
                    if ((y >> k) & 1) w = dmul(w, ptid[5 + k]);
                put(b + 36 + y, w);
            }
        }
    } else if (op.type == OP_U2) {
        const double *m = gates[op.gate].m;
        for (int k = 0; k < 16; ++k) put(rec + k, make_double2(m[2 * k], m[2 * k + 1]));
    } else {
        put(rec, op.diag_kind == DIAG_PHASE ? tabc(op.gate) : make_double2(-1.0, 0.0));
    }
}

// LDS of one block: the tile only.  Op and round descriptors, matrices and register-bit phase
// factors are read with scalar loads; the per-thread phase tables of a folded block with vector
// loads of the slot's records (a few KB, cache resident); the per-tile products of the phases
// conditioned on tile-number bits come from the table written by k_pass_jobs.

// Register tiles of 16 complex<float> or 8 complex<double> (and more) need more than 128
// VGPRs: those tiles have at most 256 threads and may use the whole register file.
template <typename R, int RB>
constexpr bool kWideTile = RB == 4 || (sizeof(R) == 8 && RB == 3);

// Waves per SIMD the register allocation must allow.  complex<float> with 16-register tiles is
// held to 128 VGPRs, so that four 256-thread blocks share a CU (their 32 KiB tiles fit the
// 160 KiB of LDS): more waves hide the tile loads and the LDS exchanges better than the
// registers the compiler would otherwise keep for scheduling.
template <typename R, int RB>
constexpr int kMinWaves = (sizeof(R) == 4 && RB == 4) ? 4 : 1;

// UNI: whether blocks whose factors do not depend on thread-id bits take their per-thread factor
// with a uniform load (the host picks this variant for passes where most blocks are such; the
// other keeps the per-thread lookups branch-free, which schedules better when few are).
// ZV: which one-qubit ops act on a target that still holds its basis bit (the zero-input
// updates): 0 none, 1 some, 2 all.  Variants 0 and 2 leave out the code paths they cannot take
// (the op dispatch of variant 1 is the largest; without it random layers measured 2-3% faster).
// ZV 3: as 2, and every one-qubit op has a real matrix, no input phase and at most a uniform
// output factor (the QFT's passes), so the op loop holds only those paths.  ZV 4: as 0, and
// every one-qubit op has a real matrix and no folded phase (Grover's Hadamard layers).  ZV 5:
// no one-qubit op at all (density-matrix passes of dense two-qubit superoperators and diagonal
// patterns).
// MIX: whether the pass has ops other than one-qubit gates (dense two-qubit gates, diagonal
// patterns left standalone); without them the op loop holds only the one-qubit paths (QFT
// and random-layer passes 1-2% faster).
template <typename R, int RB, bool UNI, bool BLK, int ZV, bool MIX>
__global__ void __launch_bounds__((kWideTile<R, RB>) ? 256 : 512)
    __attribute__((amdgpu_waves_per_eu(kMinWaves<R, RB>, 8))) k_fused(R *__restrict__ psi, int n, int S, int pass_index,
                                                  int rec_cap, int64_t init, int64_t basis, uint32_t blocal,
                                                  const RunParams *__restrict__ dyn,
                                                  const PassDesc *__restrict__ g_passes,
                                                  const StageDesc *__restrict__ g_stages,
                                                  const RoundDesc *__restrict__ g_rounds,
                                                  const OpDesc *__restrict__ g_ops,
                                                  const cxf<R> *__restrict__ rec_all,
                                                  const cxf<R> *__restrict__ wtab,
                                                  const uint64_t *__restrict__ otab,
                                                  double *__restrict__ ovl, int slot_base, int slots)
{
    // Descriptor arrays as separate read-only, non-aliasing arguments: their uniform reads
    // become scalar loads that do not wait on the tile's vector memory traffic.
    struct {
        const PassDesc *__restrict__ passes;
        const StageDesc *__restrict__ stages;
        const RoundDesc *__restrict__ rounds;
        const OpDesc *__restrict__ ops;
    } prog = {g_passes, g_stages, g_rounds, g_ops};
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NR = 1 << RB;
    const PassDesc *pd = prog.passes + pass_index;
    const int K = pd->K;
    // A run starts in the basis state |basis>, and a physical qubit no non-diagonal gate has
    // touched still holds its basis value (controlled phases only rescale), so only the tiles
    // that agree with it on the pass's classical bits hold amplitude, and inside a tile only the
    // amplitudes that agree with it on the tile-local classical bits.  A pass is launched over
    // the tiles that hold amplitude (its blocks walk the other tile-number bits) and reads only
    // those amplitudes; the first pass also stores the other tiles as zeros when no later pass
    // rewrites them.
    const bool first = init >= 0;
    if (dyn) {
        basis = dyn->init;
        if (first) init = basis;
    }
    const bool fill = first && pd->zero_fill;
    const uint64_t walk = fill ? pd->outer_mask : (pd->outer_mask & ~pd->classical);
    const int tiles_log = __builtin_popcountll(walk);
    // Block order: slot-major, so that the blocks in flight share one slot's records.  When the
    // pass also forms the overlaps with slot 0 (slots [slot_base, slot_base + slots)), tile-major
    // with the slot fastest: all slots of a tile run together and read slot 0's tile from the
    // caches.  (Measured against groups of 2^10 tiles, group-major, and against slot groups of 8
    // with one slot per XCD: both slower, as slot 0's tiles are then reused from further away.)
    int slot;
    uint64_t tile;
    if (ovl) {
        slot = slot_base + (int)(blockIdx.x % (unsigned)slots);
        tile = blockIdx.x / (unsigned)slots;
    } else {
        slot = (int)(blockIdx.x >> tiles_log);
        tile = (uint64_t)blockIdx.x & ((1ull << tiles_log) - 1ull);
    }
    // uniform by construction; the division above runs on the vector ALUs, so say so, and the
    // record and table pointers derived from them stay in scalar registers
    slot = __builtin_amdgcn_readfirstlane(slot);
    tile = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(tile >> 32)) << 32) |
           (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)tile);
    const uint64_t bidx = ((uint64_t)slot << tiles_log) | tile;
    const uint32_t tid = threadIdx.x, nthr = blockDim.x;
    const cxf<R> *__restrict__ rec = rec_all + (size_t)slot * pd->rec_size;
    // this tile's products of the phases conditioned on tile-number bits (one per outer job)
    const cxf<R> *__restrict__ wout = wtab + bidx * (size_t)(pd->job_end - pd->job_begin);

    // Outer (tile-number) bits of the physical index, written for this launch by k_pass_jobs.
    const uint64_t outer = otab[tile];
    // Load (and store) layout: the register bits are the tile-local bits of its round
    // descriptor's mask, the thread id fills the others, lowest first.  lthr0: the thread's
    // tile-local index bits in that layout (a zero bit inserted at each register bit).
    const uint32_t load_mask = prog.rounds[pd->load_round].reg_mask;
    uint64_t gthr = outer;
    uint32_t lthr0 = tid;
    {
        uint32_t m = load_mask;
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            const uint32_t b = (uint32_t)__builtin_ctz(m);
            const uint32_t lo = lthr0 & ((1u << b) - 1u);
            lthr0 = ((lthr0 ^ lo) << 1) | lo;
            m &= m - 1u;
        }
        for (int j = 0; j < K; ++j)
            if ((lthr0 >> j) & 1u) gthr |= 1ull << pd->q_pos[j];
    }
    uint64_t greg[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) greg[r] = pd->reg_off[r];
    R *base = psi + ((uint64_t)slot << (n + 1));
    // the basis index's bits at the tile-local positions (from the host, or here when the
    // basis comes from the device block)
    if (dyn) {
        blocal = 0;
        for (int j = 0; j < K; ++j)
            if (((uint64_t)basis >> pd->q_pos[j]) & 1ull) blocal |= 1u << j;
    }
    tv<R> a[NR];
    if (fill && ((outer ^ (uint64_t)basis) & pd->classical) != 0) {
        // a tile of the first pass outside the support: zeros (uniform per block)
#pragma unroll
        for (int r = 0; r < NR; ++r)
            __builtin_nontemporal_store(tv<R>{(R)0, (R)0}, reinterpret_cast<tv<R> *>(base + 2 * (gthr | greg[r])));
        if (ovl && tid < 3) ovl[bidx * 3 + tid] = 0.0;
        return;
    }
    if (init >= 0) {
        // first pass of a run: every slot starts in the basis state |init>, made here
        // instead of read from memory
#pragma unroll
        for (int r = 0; r < NR; ++r) a[r] = tv<R>{(gthr | greg[r]) == (uint64_t)init ? (R)1 : (R)0, (R)0};
    } else {
        // read only the amplitudes that can be nonzero: tile-local index lthr0 | roff[r] agrees
        // with the basis index on the tile-local classical bits (thread part per lane, register
        // part uniform)
        const uint32_t lc = pd->lclassical;
        if (lc == 0) {
#pragma unroll
            for (int r = 0; r < NR; ++r)
                a[r] = __builtin_nontemporal_load(reinterpret_cast<const tv<R> *>(base + 2 * (gthr | greg[r])));
        } else {
#pragma unroll
            for (int r = 0; r < NR; ++r) a[r] = tv<R>{(R)0, (R)0};
            // only lanes whose thread part agrees with the basis read anything, so a wave with
            // none of them (most waves when few tile bits are touched) skips the loads
            const bool tok = ((lthr0 ^ blocal) & lc & ~load_mask) == 0;
            if (tok) {
                const RoundDesc *ld = prog.rounds + pd->load_round;
#pragma unroll
                for (int r = 0; r < NR; ++r) {
                    const bool rok = ((ld->roff[r] ^ blocal) & lc & load_mask) == 0;
                    if (rok) {
                        const uint64_t i = gthr | greg[r];
                        a[r] = __builtin_nontemporal_load(reinterpret_cast<const tv<R> *>(base + 2 * i));
                    }
                }
            }
        }
    }

    // Register layout: tile-local index of register r of this thread = lthr | roff[r], with
    // roff from the current round's descriptor (cur_ri; at first the load layout's).  LDS addresses: swz(lthr | roff[r]) = swz(lthr) ^ swz(roff[r]); the register
    // part is the descriptor's sroff (one scalar load of 16 words), so each access costs one
    // XOR.  The tile sits at the start of the dynamic LDS, addressed directly.
    constexpr uint32_t CXS = sizeof(cxf<R>);
    typedef R v2 __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(3))) v2 lds_v2;
    // the kernel declares no static LDS (checked on the host before its first launch), so the
    // dynamic LDS, and the tile at its start, begins at LDS address 0
    auto lds_put = [](uint32_t byte, cxf<R> x) {
        *reinterpret_cast<lds_v2 *>((size_t)byte) = v2{x.re, x.im};
    };
    auto lds_get = [](uint32_t byte) {
        const v2 v = *reinterpret_cast<const lds_v2 *>((size_t)byte);
        return cxf<R>{v.x, v.y};
    };
    uint32_t cur = load_mask;
    // current register layout as an index into the rounds array: loads through the kernel
    // argument with a uniform index stay scalar
    int cur_ri = pd->load_round;
    uint32_t lthr = lthr0;

    auto exchange_to = [&](uint32_t to, int ri) {
        __syncthreads();
        {
            // opaque to the optimiser, which would otherwise distribute the swizzle and the
            // scaling over every access (three VALU ops per access instead of one XOR)
            uint32_t sw = swz(lthr) * CXS;
            asm volatile("" : "+v"(sw));
            const RoundDesc *from = prog.rounds + cur_ri;
#pragma unroll
            for (int r = 0; r < NR; ++r) lds_put(sw ^ (from->sroff[r] * CXS), cx<R>(a[r]));
        }
        __syncthreads();
        const RoundDesc *rd = prog.rounds + ri;
        cur = to;
        cur_ri = ri;
        // the thread id deposited into the tile-local bits outside the registers: a zero bit
        // inserted at each register bit, lowest first (arithmetic, no table load to wait on)
        {
            uint32_t x = tid, m = to;
#pragma unroll
            for (int k = 0; k < RB; ++k) {
                const uint32_t b = (uint32_t)__builtin_ctz(m);
                const uint32_t lo = x & ((1u << b) - 1u);
                x = ((x ^ lo) << 1) | lo;
                m &= m - 1u;
            }
            lthr = x;
        }
        uint32_t sw = swz(lthr) * CXS;
        asm volatile("" : "+v"(sw));
#pragma unroll
        for (int r = 0; r < NR; ++r) a[r] = tvec(lds_get(sw ^ (rd->sroff[r] * CXS)));
    };

    // A diagonal-pattern op: its tile-local condition splits into the lane's thread bits (one
    // compare per lane) and the register bits (the same for every lane), so only the registers
    // whose bits match are multiplied (a Grover sign flip on all qubits touches one of 16).
    auto diag_op = [&](const OpDesc *op) {
        const bool ohit = (outer & op->omask) == op->ovalue;
        const uint32_t lmask = op->lmask, lvalue = op->lvalue;
        const uint32_t rm = prog.rounds[cur_ri].reg_mask;
        const bool thit = ohit && (lthr & lmask) == (lvalue & ~rm);
        const uint32_t rmask = lmask & rm, rval = lvalue & rm;
        const cxf<R> f = rec[op->rec];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if ((prog.rounds[cur_ri].roff[r] & rmask) == rval) {
                const tv<R> y = tvec(mul(f, cx<R>(a[r])));
                a[r] = thit ? y : a[r];
            }
        }
    };

    for (int si = pd->stage_begin; si < pd->stage_end; ++si) {
        const StageDesc sd = prog.stages[si];
        for (int ri = sd.round_begin; ri < sd.round_end; ++ri) {
            const RoundDesc *rd = prog.rounds + ri;
            const uint32_t mask = rd->reg_mask;
            if (mask != cur) exchange_to(mask, ri);
            if constexpr (BLK && sizeof(R) == 4 && RB == 4) {
                // every round of a block pass is a block (the planner makes it all or none), so
                // this variant carries no op-by-op path
                {
                    // the round as one dense block: the ops' phases conditioned outside the
                    // registers before and after it (per op, on its target's |1> states)
                    const float *tp = reinterpret_cast<const float *>(rec + rd->block_rec) + (tid & 63u) * 16;
                    float A[16];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        const float4 q4 = *reinterpret_cast<const float4 *>(tp + 4 * k);
                        A[4 * k] = q4.x;
                        A[4 * k + 1] = q4.y;
                        A[4 * k + 2] = q4.z;
                        A[4 * k + 3] = q4.w;
                    }
                    for (int oi = rd->op_begin; oi < rd->op_end; ++oi) {
                        const OpDesc *op = prog.ops + oi;
                        const int flags = op->flags;
                        if (op->pre_rec >= 0 && (!(flags & OPF_PRE_UNI) || op->pre_job >= 0)) {
                            PhaseSet<R, RB> pre;
                            load_phases<R, RB>(pre, rec + op->pre_rec, rec + op->pre_rec, true, false,
                                               UNI && (flags & OPF_PRE_UNI) != 0, op->pre_job, wout, tid);
                            dispatch_phase_on_bit<R, RB>(op->p0, a, pre.w);
                        }
                    }
                    block_apply(a, A);
                    for (int oi = rd->op_begin; oi < rd->op_end; ++oi) {
                        const OpDesc *op = prog.ops + oi;
                        const int flags = op->flags;
                        if (op->post_rec >= 0 && (!(flags & OPF_POST_UNI) || op->post_job >= 0)) {
                            PhaseSet<R, RB> post;
                            load_phases<R, RB>(post, rec + op->post_rec, rec + op->post_rec, true, false,
                                               UNI && (flags & OPF_POST_UNI) != 0, op->post_job, wout, tid);
                            dispatch_phase_on_bit<R, RB>(op->p0, a, post.w);
                        }
                    }
                }
            } else {
            if constexpr (ZV == 3 && RB == 4) {
                // a round of untouched-target updates on register bits k-1, ..., 0: straight-line,
                // no per-op dispatch (its merges copy the register tile)
                const int seq = rd->seq;
                if (seq > 0) {
                    auto step = [&](int oi, auto pc) {
                        constexpr int PP = decltype(pc)::value;
                        const OpDesc *op = prog.ops + oi;
                        const cxf<R> *__restrict__ orec = rec + op->rec;
                        const int postr = op->post_rec, postj = op->post_job;
                        cxf<R> w = cxf<R>{(R)1, (R)0};
                        if (postr >= 0) {
                            w = rec[postr + 4];
                            if (postj >= 0) w = mul(w, wout[postj]);
                        }
                        const bool bit1 = (blocal & prog.rounds[cur_ri].roff[1 << PP]) != 0;
                        const R A = bit1 ? orec[1].re : orec[0].re;
                        const R Bm = bit1 ? orec[3].re : orec[2].re;
                        apply_u1_untouched<R, RB, PP>(a, A, cxf<R>{Bm * w.re, Bm * w.im});
                    };
                    const int ob = rd->op_begin;
                    if (seq == 4) {
                        step(ob, std::integral_constant<int, 3>{});
                        step(ob + 1, std::integral_constant<int, 2>{});
                        step(ob + 2, std::integral_constant<int, 1>{});
                        step(ob + 3, std::integral_constant<int, 0>{});
                    } else if (seq == 3) {
                        step(ob, std::integral_constant<int, 2>{});
                        step(ob + 1, std::integral_constant<int, 1>{});
                        step(ob + 2, std::integral_constant<int, 0>{});
                    } else if (seq == 2) {
                        step(ob, std::integral_constant<int, 1>{});
                        step(ob + 1, std::integral_constant<int, 0>{});
                    } else {
                        step(ob, std::integral_constant<int, 0>{});
                    }
                    continue;
                }
            }
            if constexpr (ZV == 4 && RB == 4) {
                // rounds of real updates of touched targets on register bits 0, ..., k-1 in turn
                // (seq = k), or two such runs of four around one diagonal pattern (seq = 9):
                // straight-line, the target bits fixed at compile time
                const int seq = rd->seq;
                if (seq > 0) {
                    PhaseSet<R, RB> none;
                    none.any = false;
                    auto step = [&](int oi, auto pc) {
                        constexpr int PP = decltype(pc)::value;
                        const cxf<R> *__restrict__ orec = rec + prog.ops[oi].rec;
                        const cxf<R> m[4] = {orec[0], orec[1], orec[2], orec[3]};
                        apply_u1_real<R, RB, PP, 0, 0, 0>(a, m, none, none);
                    };
                    auto run4 = [&](int ob) {
                        step(ob, std::integral_constant<int, 0>{});
                        step(ob + 1, std::integral_constant<int, 1>{});
                        step(ob + 2, std::integral_constant<int, 2>{});
                        step(ob + 3, std::integral_constant<int, 3>{});
                    };
                    const int ob = rd->op_begin;
                    if (seq == 9) {
                        run4(ob);
                        diag_op(prog.ops + ob + 4);
                        run4(ob + 5);
                    } else if (seq == 4) {
                        run4(ob);
                    } else if (seq == 3) {
                        step(ob, std::integral_constant<int, 0>{});
                        step(ob + 1, std::integral_constant<int, 1>{});
                        step(ob + 2, std::integral_constant<int, 2>{});
                    } else if (seq == 2) {
                        step(ob, std::integral_constant<int, 0>{});
                        step(ob + 1, std::integral_constant<int, 1>{});
                    } else {
                        step(ob, std::integral_constant<int, 0>{});
                    }
                    continue;
                }
            }
            const int oe = rd->op_end;
            for (int oi = rd->op_begin; oi < oe; ++oi) {
                const OpDesc *op = prog.ops + oi;
                const int type = op->type;
                const cxf<R> *__restrict__ orec = rec + op->rec;
                if (ZV == 4 && type == OP_U1) {
                    // every one-qubit op of the pass: real matrix, no folded phase, target
                    // already touched (the general pair update)
                    cxf<R> m[4] = {orec[0], orec[1], orec[2], orec[3]};
                    PhaseSet<R, RB> none;
                    none.any = false;
                    dispatch_u1_pp<R, RB, 0, 0, 0>(op->p0, true, a, m, none, none);
                } else if (ZV == 3 && type == OP_U1) {
                    // every one-qubit op of the pass: real matrix, target still untouched, no
                    // input phase, output phase at most one uniform factor
                    cxf<R> m[4] = {orec[0], orec[1], orec[2], orec[3]};
                    // an op without an output block takes the factor 1: one update path per
                    // target and input instead of two
                    PhaseSet<R, RB> pre, post;
                    pre.any = false;
                    post.any = true;
                    const int postr = op->post_rec, postj = op->post_job;
                    post.w = cxf<R>{(R)1, (R)0};
                    if (postr >= 0) {
                        post.w = rec[postr + 4];
                        if (postj >= 0) post.w = mul(post.w, wout[postj]);
                    }
                    const bool bit1 = (blocal & prog.rounds[cur_ri].roff[1 << op->p0]) != 0;
                    if (bit1) dispatch_u1_pp<R, RB, 0, 1, 2>(op->p0, true, a, m, pre, post);
                    else dispatch_u1_pp<R, RB, 0, 1, 1>(op->p0, true, a, m, pre, post);
                } else if (ZV != 5 && type == OP_U1) {
                    cxf<R> m[4] = {orec[0], orec[1], orec[2], orec[3]};
                    PhaseSet<R, RB> pre, post;
                    const int flags = op->flags;
                    const int prer = op->pre_rec, postr = op->post_rec;
                    const int prej = op->pre_job, postj = op->post_job;
                    // a target qubit no earlier gate has touched holds the basis bit: when that
                    // bit is 0 every |1> input is zero (and its input phase has nothing to do),
                    // when it is 1 every |0> input
                    const bool untouched = ZV >= 2 || (ZV == 1 && ((op->creg >> op->p0) & 1u) != 0);
                    const bool bit1 = (blocal & prog.rounds[cur_ri].roff[1 << op->p0]) != 0;
                    const bool zero_in = untouched && !bit1;
                    const int zin = untouched ? (bit1 ? 2 : 1) : 0;
                    int prekind;
                    if (zero_in) {
                        pre.any = false;
                        prekind = 0;
                    } else if (flags & OPF_UPHASE) {
                        // uniform input phase (an inner phase-chain member with no folded block)
                        pre.any = true;
                        pre.w = orec[4];
                        prekind = 1;
                    } else {
                        const bool bits = !(flags & OPF_PREW);
                        load_phases<R, RB>(pre, rec + prer, rec + prer, prer >= 0, bits,
                                           UNI && (flags & OPF_PRE_UNI) != 0, prej, wout, tid);
                        prekind = prer < 0 ? 0 : bits ? 2 : 1;
                    }
                    const bool postbits = !(flags & OPF_POSTW);
                    load_phases<R, RB>(post, rec + postr, rec + postr, postr >= 0, postbits,
                                       UNI && (flags & OPF_POST_UNI) != 0, postj, wout, tid);
                    const int postkind = postr < 0 ? 0 : postbits ? 2 : 1;
                    dispatch_u1<R, RB>(op->p0, (flags & OPF_REAL) != 0, prekind, zin, postkind, a, m, pre,
                                       post);
                } else if (MIX && type == OP_U2) {
                    cxf<R> m[16];
#pragma unroll
                    for (int k = 0; k < 16; ++k) m[k] = orec[k];
                    dispatch_u2<R, RB>(op->p0, op->p1, (op->flags & OPF_REAL) != 0, a, m);
                } else if (MIX) {
                    diag_op(op);
                }
            }
            }
        }
    }
    // Slot 0's amplitudes for the overlaps, loaded before the last exchange so that their latency
    // overlaps it (slot 0 is final before a launch of the other slots; these loads precede this
    // block's own stores).
    // The tile is stored in the pass's store layout: the last round's when the planner chose
    // it (no exchange back), else the load layout.
    const int st_ri = pd->store_round;
    uint64_t gst = gthr;
    if (st_ri != pd->load_round) {
        uint32_t x = tid, m = prog.rounds[st_ri].reg_mask;
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            const uint32_t b = (uint32_t)__builtin_ctz(m);
            const uint32_t lo = x & ((1u << b) - 1u);
            x = ((x ^ lo) << 1) | lo;
            m &= m - 1u;
        }
        gst = outer;
        for (int j = 0; j < K; ++j)
            if ((x >> j) & 1u) gst |= 1ull << pd->q_pos[j];
    }
    tv<R> refv[NR];
    const bool pre_ref = ovl != nullptr && slot != 0;
    if (pre_ref) {
#pragma unroll
        for (int r = 0; r < NR; ++r)
            refv[r] = *reinterpret_cast<const tv<R> *>(psi + 2 * (gst | pd->store_off[r]));
    }
    if (cur != prog.rounds[st_ri].reg_mask) exchange_to(prog.rounds[st_ri].reg_mask, st_ri);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        uint64_t i = gst | pd->store_off[r];
        if constexpr (sizeof(R) == 4) {
            typedef float f2 __attribute__((ext_vector_type(2)));
            __builtin_nontemporal_store(a[r], reinterpret_cast<f2 *>(base + 2 * i));
        } else {
            typedef double d2 __attribute__((ext_vector_type(2)));
            __builtin_nontemporal_store(a[r], reinterpret_cast<d2 *>(base + 2 * i));
        }
    }
    if (ovl) {
        // This tile's share of <psi_0|psi_slot> and <psi_slot|psi_slot> in FP64: the same sums
        // as the separate overlap reduction, one partial per (slot, tile).
        // Each product is one multiply-add into the running sum (for complex<float> the products
        // are exact in FP64, so this rounds once per term); the choice of reference is uniform,
        // so it is a branch rather than a select per amplitude.
        double v[3] = {0.0, 0.0, 0.0};
        if (pre_ref) {
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const double ar = refv[r].x, ai = refv[r].y, br = a[r].x, bi = a[r].y;
                v[0] = __builtin_fma(ai, bi, __builtin_fma(ar, br, v[0]));
                v[1] = __builtin_fma(-ai, br, __builtin_fma(ar, bi, v[1]));
                v[2] = __builtin_fma(bi, bi, __builtin_fma(br, br, v[2]));
            }
        } else {
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                const double br = a[r].x, bi = a[r].y;
                v[2] = __builtin_fma(bi, bi, __builtin_fma(br, br, v[2]));
            }
            v[0] = v[2];
        }
        // Block sums.  With more than one wave, every thread leaves its three sums in the LDS
        // (the tile's LDS, free once every wave has left the last exchange, holds three doubles
        // per thread when a thread keeps at least 16 bytes of amplitudes) and the first wave adds
        // them up, so the other waves finish without any cross-lane work.  A block of at most
        // one wave (or with too little LDS per thread) sums over its lanes, then over waves.
        constexpr bool kLdsSums = (sizeof(R) << (RB + 1)) >= 3 * sizeof(double);
        if (kLdsSums && nthr > 64u) {
            __syncthreads();
            double *sh = reinterpret_cast<double *>(smem);
#pragma unroll
            for (int k = 0; k < 3; ++k) sh[k * nthr + tid] = v[k];
            __syncthreads();
            if (tid < 64u) {
                double t[3] = {0.0, 0.0, 0.0};
                for (uint32_t j = tid; j < nthr; j += 64u)
#pragma unroll
                    for (int k = 0; k < 3; ++k) t[k] += sh[k * nthr + j];
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    for (int off = 32; off > 0; off >>= 1) t[k] += __shfl_xor(t[k], off, 64);
                if (tid == 0)
                    for (int k = 0; k < 3; ++k) ovl[bidx * 3 + k] = t[k];
            }
        } else {
            // wave sums (a block of fewer than 64 threads is one partial wave: sum over its lanes)
            const int width = nthr < 64u ? (int)nthr : 64;
#pragma unroll
            for (int k = 0; k < 3; ++k)
                for (int off = width >> 1; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, width);
            if (nthr <= 64u) {
                if (tid == 0)
                    for (int k = 0; k < 3; ++k) ovl[bidx * 3 + k] = v[k];
            } else {
                __syncthreads();
                double *sh = reinterpret_cast<double *>(smem);
                if ((tid & 63u) == 0)
                    for (int k = 0; k < 3; ++k) sh[(tid >> 6) * 3 + k] = v[k];
                __syncthreads();
                if (tid < 3) {
                    double t = 0.0;
                    for (uint32_t w = 0; w < (nthr >> 6); ++w) t += sh[w * 3 + tid];
                    ovl[bidx * 3 + tid] = t;
                }
            }
        }
    }
}

// Record entries per stage: 8 KiB of records (a stage bounds the descriptor ranges the kernel
// walks between two plan boundaries); 0 when the tile does not fit the 160 KiB of LDS.
int stage_rec_cap(qs_dtype dt, int K)
{
    const size_t cxs = dt == QS_C64 ? 8 : 16;
    if ((size_t(1) << K) * cxs > 160 * 1024) return 0;
    return (int)(8192 / cxs);
}

// LDS of one block: its tile.
size_t fused_lds_bytes(qs_dtype dt, int K)
{
    return (size_t(1) << K) * (dt == QS_C64 ? 8 : 16);
}

hipError_t launch_pass_prep(qs_dtype dt, int S, const PassDesc *h, ProgramDev prog,
                            const double *tab, const qs_gate *gates_dev, void *rec, int64_t basis,
                            const RunParams *dyn, hipStream_t st)
{
    const int n_ops = h->op_end - h->op_begin;
    const uint64_t tot = (uint64_t)n_ops * S;
    if (tot == 0) return hipSuccess;
    TimedLaunch tl("prep", (double)S * h->rec_size * (dt == QS_C64 ? 8 : 16), st);
    unsigned blocks = (unsigned)((tot + 127) / 128);
    if (dt == QS_C64)
        hipLaunchKernelGGL(k_pass_prep<float>, dim3(blocks), dim3(128), 0, st, S, h->op_begin, n_ops,
                           h->rec_size, prog, tab, gates_dev, (cxf<float> *)rec, (uint64_t)basis, dyn);
    else
        hipLaunchKernelGGL(k_pass_prep<double>, dim3(blocks), dim3(128), 0, st, S, h->op_begin, n_ops,
                           h->rec_size, prog, tab, gates_dev, (cxf<double> *)rec, (uint64_t)basis, dyn);
    return hipGetLastError();
}

hipError_t launch_block_prep(qs_dtype dt, int S, const PassDesc *h, ProgramDev prog, void *rec, hipStream_t st)
{
    const int n_rounds = h->round_end - h->round_begin;
    const int64_t tot = (int64_t)S * n_rounds * 16;
    if (tot == 0 || dt != QS_C64) return hipSuccess;
    TimedLaunch tl("prep", (double)S * n_rounds * kBlockRecEntries * 8.0, st);
    hipLaunchKernelGGL(k_block_prep<float>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, S, h->round_begin,
                       n_rounds, h->rec_size, prog, (cxf<float> *)rec);
    return hipGetLastError();
}

hipError_t launch_pass_jobs(qs_dtype dt, int n, int S, const PassDesc *h, ProgramDev prog, const void *rec,
                            int64_t init, int64_t basis, const RunParams *dyn, void *wtab, uint64_t *otab,
                            hipStream_t st)
{
    const int n_jobs = h->job_end - h->job_begin;
    const bool fill = init >= 0 && h->zero_fill;
    const uint64_t walk = fill ? h->outer_mask : (h->outer_mask & ~h->classical);
    const int tiles_log = __builtin_popcountll(walk);
    const uint64_t classical = fill ? 0 : h->classical;
    const uint64_t fixed_bits = (uint64_t)basis & classical;
    const int64_t tot = ((int64_t)S << tiles_log) * (n_jobs > 0 ? n_jobs : 1);
    TimedLaunch tl("jobs", (double)((int64_t)S << tiles_log) * n_jobs * (dt == QS_C64 ? 8 : 16), st);
    const unsigned blocks = (unsigned)((tot + 255) / 256);
    if (dt == QS_C64)
        hipLaunchKernelGGL(k_pass_jobs<float>, dim3(blocks), dim3(256), 0, st, S, n_jobs, tiles_log, walk, fixed_bits,
                           h->rec_size, prog.jobs + h->job_begin, prog.obits, (const cxf<float> *)rec, dyn,
                           classical, (cxf<float> *)wtab, otab);
    else
        hipLaunchKernelGGL(k_pass_jobs<double>, dim3(blocks), dim3(256), 0, st, S, n_jobs, tiles_log, walk,
                           fixed_bits, h->rec_size, prog.jobs + h->job_begin, prog.obits, (const cxf<double> *)rec,
                           dyn, classical, (cxf<double> *)wtab, otab);
    return hipGetLastError();
}

// thread-safe one-time opt-in to the full 160 KiB of LDS
template <typename R, int RB, bool UNI, bool BLK, int ZV, bool MIX>
static hipError_t fused_attr_one()
{
    static const hipError_t attr = [] {
        // the kernel addresses its tile at LDS address 0: it must have no static LDS
        hipFuncAttributes fa;
        hipError_t e = hipFuncGetAttributes(&fa, (const void *)k_fused<R, RB, UNI, BLK, ZV, MIX>);
        if (e != hipSuccess) return e;
        if (fa.sharedSizeBytes != 0) return hipErrorInvalidKernelFile;
        return hipFuncSetAttribute((const void *)k_fused<R, RB, UNI, BLK, ZV, MIX>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    }();
    return attr;
}

template <typename R, int RB, bool UNI, int ZV>
static hipError_t fused_attr_mix()
{
    hipError_t e = fused_attr_one<R, RB, UNI, false, ZV, false>();
    if (e == hipSuccess) e = fused_attr_one<R, RB, UNI, false, ZV, true>();
    return e;
}

// the block-round variants (matrix-core rounds) exist for complex<float> with 16 registers only
template <typename R, int RB>
constexpr bool kBlockVariant = sizeof(R) == 4 && RB == 4;

template <typename R, int RB>
static hipError_t fused_attr()
{
    hipError_t e = fused_attr_mix<R, RB, false, 0>();
    if (e == hipSuccess) e = fused_attr_mix<R, RB, true, 0>();
    if (e == hipSuccess) e = fused_attr_mix<R, RB, false, 1>();
    if (e == hipSuccess) e = fused_attr_mix<R, RB, true, 1>();
    if (e == hipSuccess) e = fused_attr_mix<R, RB, false, 2>();
    if (e == hipSuccess) e = fused_attr_mix<R, RB, true, 2>();
    if (e == hipSuccess) e = fused_attr_one<R, RB, true, false, 3, false>();
    if (e == hipSuccess) e = fused_attr_mix<R, RB, false, 4>();
    if (e == hipSuccess) e = fused_attr_one<R, RB, false, false, 5, true>();
    if constexpr (kBlockVariant<R, RB>) {
        // block rounds replace the op-by-op loop: no zero-input paths there
        if (e == hipSuccess) e = fused_attr_one<R, RB, false, true, 0, true>();
        if (e == hipSuccess) e = fused_attr_one<R, RB, true, true, 0, true>();
    }
    return e;
}

hipError_t fused_prepare_attributes()
{
    hipError_t e;
    if ((e = fused_attr<float, 1>()) != hipSuccess || (e = fused_attr<float, 2>()) != hipSuccess ||
        (e = fused_attr<float, 3>()) != hipSuccess || (e = fused_attr<float, 4>()) != hipSuccess ||
        (e = fused_attr<double, 1>()) != hipSuccess || (e = fused_attr<double, 2>()) != hipSuccess ||
        (e = fused_attr<double, 3>()) != hipSuccess || (e = fused_attr<double, 4>()) != hipSuccess)
        return e;
    return hipSuccess;
}

template <typename R, int RB>
static hipError_t launch_t(R *psi, int n, int S, const PassDesc &h, int pass_index, int rec_cap,
                           int64_t init, int64_t basis, const RunParams *dyn, ProgramDev prog, const void *rec,
                           const void *wtab, const uint64_t *otab, size_t lds, hipStream_t st,
                           double *ovl, int slot_base, int slots)
{
    const hipError_t attr = fused_attr<R, RB>();
    if (attr != hipSuccess) return attr;
    // the first pass may store every tile; otherwise a pass runs over the tiles that hold amplitude
    const bool fill = init >= 0 && h.zero_fill;
    const int free_bits = n - h.K - (fill ? 0 : __builtin_popcountll(h.classical));
    unsigned blocks = (unsigned)((uint64_t)(ovl ? slots : S) << free_bits);
    unsigned threads = 1u << (h.K - RB);
    uint32_t blocal = 0;
    for (int j = 0; j < h.K; ++j)
        if (((uint64_t)basis >> h.q_pos[j]) & 1ull) blocal |= 1u << j;
#define QS_FUSED_LAUNCH_M(UNI, BLK, ZV, MIX)                                                                   \
    hipLaunchKernelGGL((k_fused<R, RB, UNI, BLK, ZV, MIX>), dim3(blocks), dim3(threads), lds, st, psi, n, S, pass_index, \
                       rec_cap, init, basis, blocal, dyn, prog.passes, prog.stages, prog.rounds, prog.ops,         \
                       (const cxf<R> *)rec, (const cxf<R> *)wtab, otab, ovl, slot_base, slots)
#define QS_FUSED_LAUNCH(UNI, ZV)                                                                               \
    do {                                                                                                       \
        if (h.mixed_ops) QS_FUSED_LAUNCH_M(UNI, false, ZV, true);                                              \
        else QS_FUSED_LAUNCH_M(UNI, false, ZV, false);                                                         \
    } while (0)
    if constexpr (kBlockVariant<R, RB>) {
        if (h.blocks) {
            // block rounds: one variant, every op path kept
            if (h.uni_kernel) QS_FUSED_LAUNCH_M(true, true, 0, true);
            else QS_FUSED_LAUNCH_M(false, true, 0, true);
            return hipGetLastError();
        }
    }
    if (h.blocks) return hipErrorInvalidValue;   // no block-round variant for this tile shape
    if (h.zin_ops == 3) {
        QS_FUSED_LAUNCH_M(true, false, 3, false);
    } else if (h.zin_ops == 4) {
        QS_FUSED_LAUNCH(false, 4);
    } else if (h.zin_ops == 5) {
        QS_FUSED_LAUNCH_M(false, false, 5, true);
    } else if (h.zin_ops == 2) {
        if (h.uni_kernel) QS_FUSED_LAUNCH(true, 2);
        else QS_FUSED_LAUNCH(false, 2);
    } else if (h.zin_ops == 1) {
        if (h.uni_kernel) QS_FUSED_LAUNCH(true, 1);
        else QS_FUSED_LAUNCH(false, 1);
    } else {
        if (h.uni_kernel) QS_FUSED_LAUNCH(true, 0);
        else QS_FUSED_LAUNCH(false, 0);
    }
#undef QS_FUSED_LAUNCH
#undef QS_FUSED_LAUNCH_M
    return hipGetLastError();
}

int fused_walked_bits(int n, const PassDesc *pass_host, int64_t init)
{
    const bool fill = init >= 0 && pass_host->zero_fill;
    return n - pass_host->K - (fill ? 0 : __builtin_popcountll(pass_host->classical));
}

hipError_t launch_fused_pass(void *psi, qs_dtype dt, int n, int S, const PassDesc *pass_host,
                             int pass_index, int64_t init, int64_t basis, ProgramDev prog, const void *rec,
                             const void *wtab, const uint64_t *otab, hipStream_t st, const RunParams *dyn,
                             double *ovl, int slot_base, int slots)
{
    const PassDesc &h = *pass_host;
    size_t lds = fused_lds_bytes(dt, h.K);
    const int rec_cap = stage_rec_cap(dt, h.K);
    if (lds > 160 * 1024 || rec_cap <= 0 || basis < 0) return hipErrorInvalidValue;
    if (ovl && (slots < 1 || slot_base < 0 || slot_base + slots > S)) return hipErrorInvalidValue;
    const int S_run = ovl ? slots : S;
    // Algorithmic bytes: a pass writes the tiles that can hold amplitude (a 2^-popcount(classical)
    // share; every tile when the first pass stores the zeros) and reads, except the first pass,
    // the amplitudes of the support inside them (a further 2^-popcount(lclassical) share).
    const bool fill_all = init >= 0 && h.zero_fill;
    const double tiles_share = fill_all ? 1.0 : std::ldexp(1.0, -__builtin_popcountll(h.classical));
    const double read_share = init >= 0 ? 0.0 : std::ldexp(1.0, -__builtin_popcount(h.lclassical));
    // with the overlaps: slot 0's tiles once more (read from HBM once, by the first slot of a tile)
    const double ref_share = ovl && slot_base > 0 ? 1.0 : 0.0;
    TimedLaunch tl("fused",
                   ((1.0 + read_share) * (double)S_run + ref_share) * tiles_share * std::ldexp(1.0, n) * amp_bytes(dt),
                   st);
    if (dt == QS_C64) {
        float *p = (float *)psi;
        switch (h.RB) {
        case 1: return launch_t<float, 1>(p, n, S, h, pass_index, rec_cap, init, basis, dyn, prog, rec, wtab, otab, lds, st, ovl, slot_base, slots);
        case 2: return launch_t<float, 2>(p, n, S, h, pass_index, rec_cap, init, basis, dyn, prog, rec, wtab, otab, lds, st, ovl, slot_base, slots);
        case 3: return launch_t<float, 3>(p, n, S, h, pass_index, rec_cap, init, basis, dyn, prog, rec, wtab, otab, lds, st, ovl, slot_base, slots);
        case 4: return launch_t<float, 4>(p, n, S, h, pass_index, rec_cap, init, basis, dyn, prog, rec, wtab, otab, lds, st, ovl, slot_base, slots);
        }
    } else {
        double *p = (double *)psi;
        switch (h.RB) {
        case 1: return launch_t<double, 1>(p, n, S, h, pass_index, rec_cap, init, basis, dyn, prog, rec, wtab, otab, lds, st, ovl, slot_base, slots);
        case 2: return launch_t<double, 2>(p, n, S, h, pass_index, rec_cap, init, basis, dyn, prog, rec, wtab, otab, lds, st, ovl, slot_base, slots);
        case 3: return launch_t<double, 3>(p, n, S, h, pass_index, rec_cap, init, basis, dyn, prog, rec, wtab, otab, lds, st, ovl, slot_base, slots);
        case 4: return launch_t<double, 4>(p, n, S, h, pass_index, rec_cap, init, basis, dyn, prog, rec, wtab, otab, lds, st, ovl, slot_base, slots);
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace qs
