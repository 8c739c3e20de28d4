/*
 * CPU FP64 oracle for the noisy state-vector and density-matrix method of
 * Bogdanov, Chernyavskiy et al., "Numerical and analytical research of the impact of
 * decoherence on quantum circuits" (arXiv:1412.2293).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference that the
 * HIP library is checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no code with the HIP library.
 *
 * Everything here is plain loops over double-precision complex numbers, in the order the
 * paper states the operations:
 *   - Section 2: a one-qubit gate updates every amplitude pair (a_{..0..}, a_{..1..}) that
 *     differs in the target bit; multi-qubit gates likewise on 4-tuples.
 *   - Section 2, eq. (1): the Monte Carlo noisy gate is U * V(e*xi), V = [[c, s], [-s, c]],
 *     c = cos(e*xi), s = sin(e*xi), xi ~ N(0,1).
 *   - Section 2, after eq. (2): the noisy controlled phase replaces theta by theta + e*xi.
 *   - Section 3: rho is stored as the vector sum rho_ij |i>|j>; a Kraus channel is
 *     sum_k E_k rho E_k^dagger (eq. 3) with the sets of eq. (6) and eq. (9).
 *
 * Readings where the paper is silent:
 *   - qubit q is bit q of the amplitude index;
 *   - vec(rho) index = i * 2^n + j for rho_ij (ket bits high, bra bits low);
 *   - the Kraus operators of a noisy gate U are U * E_k (noise acts first, as in eq. (5));
 *   - xi is drawn by Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) with counter
 *     (site, trajectory, stream, request) and key (seed low word, seed high word), and the
 *     cosine branch of the Box-Muller transform (Box & Muller 1958).
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared (no fast-math, no contraction:
 * the normal deviates must be reproducible bit for bit).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ------------------------------------------------------------------------------------ */
/* Philox4x32-10: 10 rounds of the 4x32 Philox bijection.  Each round multiplies words 0  */
/* and 2 by the round multipliers, and the high halves of the products are xor-ed with     */
/* words 1 and 3 and the round key; the key is advanced by the Weyl constants between      */
/* rounds.                                                                                  */
/* ------------------------------------------------------------------------------------ */
#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void or_philox_batch(int64_t count, const uint32_t *ctrs, const uint32_t *keys, uint32_t *out)
{
    for (int64_t i = 0; i < count; ++i)
        or_philox4x32_10(ctrs + 4 * i, keys + 2 * i, out + 4 * i);
}

/* ------------------------------------------------------------------------------------ */
/* Natural logarithm from its definition by series: x = m * 2^k with m in [1/sqrt2,      */
/* sqrt2), log m = 2 atanh(s), s = (m-1)/(m+1), atanh s = sum s^(2j+1)/(2j+1).  |s| <=    */
/* 0.1716, so twelve terms reach far below double rounding.  Only IEEE +,-,*,/ are used,  */
/* each correctly rounded, so the result is a fixed function of x.  Valid for positive    */
/* normal x (the Box-Muller input is in [2^-53, 1]).                                       */
/* ------------------------------------------------------------------------------------ */
static const double OR_LN2_HI = 0x1.62e42fee00000p-1; /* ln 2 rounded to 32 significant bits */
static const double OR_LN2_LO = 0x1.a39ef35793c76p-33; /* ln 2 - OR_LN2_HI */
static const double OR_SQRT2 = 0x1.6a09e667f3bcdp+0;

double or_log(double x)
{
    uint64_t bits;
    memcpy(&bits, &x, sizeof bits);
    int k = (int)((bits >> 52) & 0x7ff) - 1023;
    bits = (bits & 0x000fffffffffffffull) | 0x3ff0000000000000ull;
    double m;
    memcpy(&m, &bits, sizeof m);
    if (m > OR_SQRT2) {
        m = m * 0.5;
        k = k + 1;
    }
    double s = (m - 1.0) / (m + 1.0);
    double z = s * s;
    double p = 1.0 / 23.0;
    p = p * z + 1.0 / 21.0;
    p = p * z + 1.0 / 19.0;
    p = p * z + 1.0 / 17.0;
    p = p * z + 1.0 / 15.0;
    p = p * z + 1.0 / 13.0;
    p = p * z + 1.0 / 11.0;
    p = p * z + 1.0 / 9.0;
    p = p * z + 1.0 / 7.0;
    p = p * z + 1.0 / 5.0;
    p = p * z + 1.0 / 3.0;
    p = p * z + 1.0;
    double r = 2.0 * s * p;
    double dk = (double)k;
    return dk * OR_LN2_HI + (dk * OR_LN2_LO + r);
}

/* Taylor polynomials of cos and sin on [0, pi/4], coefficients 1/(2j)! and 1/(2j+1)!. */
static double or_cos_poly(double x)
{
    double z = x * x;
    double p = 1.0 / 2432902008176640000.0;      /* 1/20! */
    p = p * z - 1.0 / 6402373705728000.0;        /* 1/18! */
    p = p * z + 1.0 / 20922789888000.0;          /* 1/16! */
    p = p * z - 1.0 / 87178291200.0;             /* 1/14! */
    p = p * z + 1.0 / 479001600.0;               /* 1/12! */
    p = p * z - 1.0 / 3628800.0;                 /* 1/10! */
    p = p * z + 1.0 / 40320.0;                   /* 1/8!  */
    p = p * z - 1.0 / 720.0;                     /* 1/6!  */
    p = p * z + 1.0 / 24.0;                      /* 1/4!  */
    p = p * z - 1.0 / 2.0;                       /* 1/2!  */
    return p * z + 1.0;
}

static double or_sin_poly(double x)
{
    double z = x * x;
    double p = -1.0 / 121645100408832000.0;      /* -1/19! */
    p = p * z + 1.0 / 355687428096000.0;         /*  1/17! */
    p = p * z - 1.0 / 1307674368000.0;           /* -1/15! */
    p = p * z + 1.0 / 6227020800.0;              /*  1/13! */
    p = p * z - 1.0 / 39916800.0;                /* -1/11! */
    p = p * z + 1.0 / 362880.0;                  /*  1/9!  */
    p = p * z - 1.0 / 5040.0;                    /* -1/7!  */
    p = p * z + 1.0 / 120.0;                     /*  1/5!  */
    p = p * z - 1.0 / 6.0;                       /* -1/3!  */
    return x + x * (p * z);
}

/* cos(2*pi*u) for u in [0, 1), by symmetry reduced to an argument in [0, pi/4].  u is a   */
/* multiple of 2^-53, so 1-u, 1/4-v and 1/2-v below are exact.                             */
static const double OR_TWO_PI = 0x1.921fb54442d18p+2;

double or_cos2pi(double u)
{
    double v = (u >= 0.5) ? 1.0 - u : u;          /* cos(2 pi u) = cos(2 pi (1-u)) */
    if (v <= 0.125)
        return or_cos_poly(OR_TWO_PI * v);
    if (v <= 0.375)
        return or_sin_poly(OR_TWO_PI * (0.25 - v)); /* cos(2 pi v) = sin(2 pi (1/4 - v)) */
    return -or_cos_poly(OR_TWO_PI * (0.5 - v));     /* cos(2 pi v) = -cos(2 pi (1/2 - v)) */
}

/* One N(0,1) deviate from the four Philox words: the first two give u1 in (0, 1], the last  */
/* two give u2 in [0, 1), each with 53 random bits; xi = sqrt(-2 ln u1) cos(2 pi u2).        */
double or_normal_from_words(const uint32_t w[4])
{
    uint64_t a = (((uint64_t)w[0] << 32) | (uint64_t)w[1]) >> 11;
    uint64_t b = (((uint64_t)w[2] << 32) | (uint64_t)w[3]) >> 11;
    double u1 = ((double)a + 1.0) * 0x1.0p-53;
    double u2 = (double)b * 0x1.0p-53;
    return sqrt(-2.0 * or_log(u1)) * or_cos2pi(u2);
}

double or_normal(uint64_t seed, uint32_t site, uint32_t traj, uint32_t stream, uint32_t request)
{
    uint32_t ctr[4] = {site, traj, stream, request};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    or_philox4x32_10(ctr, key, w);
    return or_normal_from_words(w);
}

/* out[t * n_sites + s] = xi for (sites[s], trajs[t]) on noise stream `stream`. */
void or_normals(uint64_t seed, uint32_t request, uint32_t stream, int64_t n_sites,
                const uint32_t *sites, int64_t n_traj, const uint32_t *trajs, double *out)
{
    for (int64_t t = 0; t < n_traj; ++t)
        for (int64_t s = 0; s < n_sites; ++s)
            out[t * n_sites + s] = or_normal(seed, sites[s], trajs[t], stream, request);
}

/* ------------------------------------------------------------------------------------ */
/* State-vector level (Section 2).                                                       */
/* ------------------------------------------------------------------------------------ */
enum { K_U1 = 0, K_CP = 1, K_SWAP = 2, K_CNOT = 3, K_U2 = 4, K_FLIP = 5, K_DIAG = 6 };
enum { N_NONE = 0, N_ROT = 1, N_PHASE = 2 };

/* b_{..0..} = u00 a_{..0..} + u01 a_{..1..},  b_{..1..} = u10 a_{..0..} + u11 a_{..1..} */
static void sv_apply_1q(cplx *psi, int n, int q, const cplx u[2][2])
{
    uint64_t N = 1ull << n, bit = 1ull << q;
    for (uint64_t i = 0; i < N; ++i) {
        if (i & bit)
            continue;
        cplx a0 = psi[i], a1 = psi[i | bit];
        psi[i] = u[0][0] * a0 + u[0][1] * a1;
        psi[i | bit] = u[1][0] * a0 + u[1][1] * a1;
    }
}

/* 4x4 gate on (qa, qb) with local index bit(qa) + 2 bit(qb). */
static void sv_apply_2q(cplx *psi, int n, int qa, int qb, const cplx u[4][4])
{
    uint64_t N = 1ull << n, ba = 1ull << qa, bb = 1ull << qb;
    for (uint64_t i = 0; i < N; ++i) {
        if ((i & ba) || (i & bb))
            continue;
        uint64_t idx[4] = {i, i | ba, i | bb, i | ba | bb};
        cplx a[4], b[4];
        for (int r = 0; r < 4; ++r)
            a[r] = psi[idx[r]];
        for (int r = 0; r < 4; ++r) {
            b[r] = 0;
            for (int c = 0; c < 4; ++c)
                b[r] += u[r][c] * a[c];
        }
        for (int r = 0; r < 4; ++r)
            psi[idx[r]] = b[r];
    }
}

static void sv_phase_11(cplx *psi, int n, int qa, int qb, cplx ph)
{
    uint64_t N = 1ull << n, m = (1ull << qa) | (1ull << qb);
    for (uint64_t i = 0; i < N; ++i)
        if ((i & m) == m)
            psi[i] *= ph;
}

static void sv_swap(cplx *psi, int n, int qa, int qb)
{
    uint64_t N = 1ull << n, ba = 1ull << qa, bb = 1ull << qb;
    for (uint64_t i = 0; i < N; ++i) {
        if ((i & ba) && !(i & bb)) {
            uint64_t j = (i & ~ba) | bb;
            cplx t = psi[i];
            psi[i] = psi[j];
            psi[j] = t;
        }
    }
}

static void sv_cnot(cplx *psi, int n, int qc, int qt)
{
    uint64_t N = 1ull << n, bc = 1ull << qc, bt = 1ull << qt;
    for (uint64_t i = 0; i < N; ++i) {
        if ((i & bc) && !(i & bt)) {
            cplx t = psi[i];
            psi[i] = psi[i | bt];
            psi[i | bt] = t;
        }
    }
}

static void sv_flip(cplx *psi, int n, uint64_t mask, uint64_t value)
{
    uint64_t N = 1ull << n;
    for (uint64_t i = 0; i < N; ++i)
        if ((i & mask) == value)
            psi[i] = -psi[i];
}

/* The diagonal gate D = I + (f - 1) sum_{i & mask == value} |i><i|. */
static void sv_diag(cplx *psi, int n, uint64_t mask, uint64_t value, cplx f)
{
    uint64_t N = 1ull << n;
    for (uint64_t i = 0; i < N; ++i)
        if ((i & mask) == value)
            psi[i] *= f;
}

static void load_u1(const double *m, cplx u[2][2])
{
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c)
            u[r][c] = m[2 * (2 * r + c)] + I * m[2 * (2 * r + c) + 1];
}

static void load_u2(const double *m, cplx u[4][4])
{
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c)
            u[r][c] = m[2 * (4 * r + c)] + I * m[2 * (4 * r + c) + 1];
}

/* Circuit in flat arrays; mats holds 32 doubles per gate (a 4x4 complex matrix, re/im     */
/* interleaved, row-major; a 2x2 uses the first 8).                                        */
typedef struct {
    int64_t n_gates;
    const int32_t *kind, *q0, *q1, *noise;
    const uint32_t *site;
    const double *mats, *theta;
    const uint64_t *mask, *value;
} or_circuit;

/* Apply the circuit to psi, one gate at a time, drawing xi for every noisy gate of         */
/* trajectory `traj`.  e = 0 gives the ideal circuit (no draws are made).                  */
static void sv_run_circuit(cplx *psi, int n, const or_circuit *c, double e, uint64_t seed,
                           uint32_t request, uint32_t traj)
{
    for (int64_t g = 0; g < c->n_gates; ++g) {
        const double *m = c->mats + 32 * g;
        int noisy = (e != 0.0) && (c->noise[g] != N_NONE);
        switch (c->kind[g]) {
        case K_U1: {
            cplx u[2][2];
            load_u1(m, u);
            if (noisy && c->noise[g] == N_ROT) {
                double xi = or_normal(seed, c->site[g], traj, 0, request);
                double cs = cos(e * xi), sn = sin(e * xi);
                cplx v[2][2] = {{cs, sn}, {-sn, cs}};
                cplx uv[2][2];
                for (int r = 0; r < 2; ++r)
                    for (int k = 0; k < 2; ++k)
                        uv[r][k] = u[r][0] * v[0][k] + u[r][1] * v[1][k];
                sv_apply_1q(psi, n, c->q0[g], (const cplx(*)[2])uv);
            } else {
                sv_apply_1q(psi, n, c->q0[g], (const cplx(*)[2])u);
            }
            break;
        }
        case K_CP: {
            double ang = c->theta[g];
            if (noisy && c->noise[g] == N_PHASE)
                ang = ang + e * or_normal(seed, c->site[g], traj, 0, request);
            sv_phase_11(psi, n, c->q0[g], c->q1[g], cos(ang) - I * sin(ang));
            break;
        }
        case K_SWAP:
            sv_swap(psi, n, c->q0[g], c->q1[g]);
            break;
        case K_CNOT:
            sv_cnot(psi, n, c->q0[g], c->q1[g]);
            break;
        case K_U2: {
            cplx u[4][4];
            load_u2(m, u);
            sv_apply_2q(psi, n, c->q0[g], c->q1[g], (const cplx(*)[4])u);
            break;
        }
        case K_FLIP:
            sv_flip(psi, n, c->mask[g], c->value[g]);
            break;
        case K_DIAG:
            sv_diag(psi, n, c->mask[g], c->value[g], m[0] + I * m[1]);
            break;
        default:
            break;
        }
    }
}

/* Apply the circuit (trajectory `traj`) to the state in psi_inout (2N doubles). */
int or_sv_apply_circuit(int n, int64_t n_gates, const int32_t *kind, const int32_t *q0,
                        const int32_t *q1, const int32_t *noise, const uint32_t *site,
                        const double *mats, const double *theta, const uint64_t *mask,
                        const uint64_t *value, double e, uint64_t seed, uint32_t request,
                        uint32_t traj, double *psi_inout)
{
    if (n < 1 || n > 34)
        return -1;
    or_circuit c = {n_gates, kind, q0, q1, noise, site, mats, theta, mask, value};
    sv_run_circuit((cplx *)psi_inout, n, &c, e, seed, request, traj);
    return 0;
}

/* |init><init| through the circuit for trajectory `traj`; psi_out holds 2N doubles. */
int or_sv_run(int n, int64_t n_gates, const int32_t *kind, const int32_t *q0, const int32_t *q1,
              const int32_t *noise, const uint32_t *site, const double *mats, const double *theta,
              const uint64_t *mask, const uint64_t *value, double e, uint64_t seed,
              uint32_t request, uint32_t traj, uint64_t init_index, double *psi_out)
{
    if (n < 1 || n > 34)
        return -1;
    uint64_t N = 1ull << n;
    if (init_index >= N)
        return -1;
    memset(psi_out, 0, sizeof(double) * 2 * N);
    psi_out[2 * init_index] = 1.0;
    return or_sv_apply_circuit(n, n_gates, kind, q0, q1, noise, site, mats, theta, mask, value,
                               e, seed, request, traj, psi_out);
}

/* <a|b> summed in index order, plus both squared norms. */
void or_inner(int64_t N, const double *a, const double *b, double *re, double *im,
              double *na, double *nb)
{
    const cplx *pa = (const cplx *)a, *pb = (const cplx *)b;
    cplx s = 0;
    double sa = 0, sb = 0;
    for (int64_t i = 0; i < N; ++i) {
        s += conj(pa[i]) * pb[i];
        sa += creal(pa[i]) * creal(pa[i]) + cimag(pa[i]) * cimag(pa[i]);
        sb += creal(pb[i]) * creal(pb[i]) + cimag(pb[i]) * cimag(pb[i]);
    }
    *re = creal(s);
    *im = cimag(s);
    *na = sa;
    *nb = sb;
}

/* ------------------------------------------------------------------------------------ */
/* Density-matrix level (Section 3).  rho_ij sits at index i*2^n + j.  E rho E^dagger is  */
/* E applied to the ket bits and conj(E) applied to the bra bits of the 2n-bit vector.    */
/* ------------------------------------------------------------------------------------ */

/* acc += E rho E^dagger for one operator E on k = 1 or 2 qubits. */
static void dm_sandwich_add(cplx *acc, const cplx *rho, cplx *tmp, int n, int k,
                            const int *qs, const cplx *E)
{
    uint64_t D = 1ull << (2 * n);
    memcpy(tmp, rho, sizeof(cplx) * D);
    if (k == 1) {
        cplx u[2][2], uc[2][2];
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 2; ++c) {
                u[r][c] = E[2 * r + c];
                uc[r][c] = conj(E[2 * r + c]);
            }
        sv_apply_1q(tmp, 2 * n, qs[0] + n, (const cplx(*)[2])u);
        sv_apply_1q(tmp, 2 * n, qs[0], (const cplx(*)[2])uc);
    } else {
        cplx u[4][4], uc[4][4];
        for (int r = 0; r < 4; ++r)
            for (int c = 0; c < 4; ++c) {
                u[r][c] = E[4 * r + c];
                uc[r][c] = conj(E[4 * r + c]);
            }
        sv_apply_2q(tmp, 2 * n, qs[0] + n, qs[1] + n, (const cplx(*)[4])u);
        sv_apply_2q(tmp, 2 * n, qs[0], qs[1], (const cplx(*)[4])uc);
    }
    for (uint64_t i = 0; i < D; ++i)
        acc[i] += tmp[i];
}

/* rho <- sum_k E_k rho E_k^dagger (eq. 3).  ops: n_ops matrices of 2^k x 2^k complex,    */
/* re/im interleaved, row-major; for k = 2 the local index is bit(q[0]) + 2 bit(q[1]).      */
int or_dm_apply_kraus(int n, double *rho, int k, const int32_t *qs, int n_ops, const double *ops)
{
    if (n < 1 || n > 14 || (k != 1 && k != 2) || n_ops < 1)
        return -1;
    uint64_t D = 1ull << (2 * n);
    int d = 1 << k;
    cplx *acc = calloc(D, sizeof(cplx));
    cplx *tmp = malloc(sizeof(cplx) * D);
    cplx *E = malloc(sizeof(cplx) * d * d);
    if (!acc || !tmp || !E) {
        free(acc); free(tmp); free(E);
        return -2;
    }
    int q[2] = {qs[0], k == 2 ? qs[1] : 0};
    for (int o = 0; o < n_ops; ++o) {
        for (int i = 0; i < d * d; ++i)
            E[i] = ops[2 * (o * d * d + i)] + I * ops[2 * (o * d * d + i) + 1];
        dm_sandwich_add(acc, (const cplx *)rho, tmp, n, k, q, E);
    }
    memcpy(rho, acc, sizeof(cplx) * D);
    free(acc); free(tmp); free(E);
    return 0;
}

/* Kraus operators of the noisy gates, eq. (6) and eq. (9), each multiplied on the left by   */
/* the ideal gate.                                                                          */
static void kraus_rot(const cplx u[2][2], double e, cplx out[2][4])
{
    double l1 = 0.5 * (1.0 + exp(-2.0 * e * e));
    double l2 = 0.5 * (1.0 - exp(-2.0 * e * e));
    cplx E1[2][2] = {{sqrt(l1), 0}, {0, sqrt(l1)}};
    cplx E2[2][2] = {{0, sqrt(l2)}, {-sqrt(l2), 0}};
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) {
            out[0][2 * r + c] = u[r][0] * E1[0][c] + u[r][1] * E1[1][c];
            out[1][2 * r + c] = u[r][0] * E2[0][c] + u[r][1] * E2[1][c];
        }
}

static void ops_to_doubles(const cplx *ops, int count, double *out)
{
    for (int i = 0; i < count; ++i) {
        out[2 * i] = creal(ops[i]);
        out[2 * i + 1] = cimag(ops[i]);
    }
}

/* Exact density-matrix run of the circuit from |init><init|, noisy gates as Kraus channels. */
int or_dm_run(int n, int64_t n_gates, const int32_t *kind, const int32_t *q0, const int32_t *q1,
              const int32_t *noise, const double *mats, const double *theta,
              const uint64_t *mask, const uint64_t *value, double e, uint64_t init_index,
              double *rho_out)
{
    if (n < 1 || n > 14)
        return -1;
    uint64_t N = 1ull << n, D = N * N;
    if (init_index >= N)
        return -1;
    memset(rho_out, 0, sizeof(double) * 2 * D);
    rho_out[2 * (init_index * N + init_index)] = 1.0;
    cplx *rho = (cplx *)rho_out;
    double buf[2 * 2 * 16];
    for (int64_t g = 0; g < n_gates; ++g) {
        const double *m = mats + 32 * g;
        int noisy = (e != 0.0) && (noise[g] != N_NONE);
        int st = 0;
        switch (kind[g]) {
        case K_U1: {
            cplx u[2][2];
            load_u1(m, u);
            int32_t q = q0[g];
            if (noisy && noise[g] == N_ROT) {
                cplx ks[2][4];
                kraus_rot((const cplx(*)[2])u, e, ks);
                ops_to_doubles(&ks[0][0], 8, buf);
                st = or_dm_apply_kraus(n, rho_out, 1, &q, 2, buf);
            } else {
                ops_to_doubles(&u[0][0], 4, buf);
                st = or_dm_apply_kraus(n, rho_out, 1, &q, 1, buf);
            }
            break;
        }
        case K_CP: {
            cplx ph = cos(theta[g]) - I * sin(theta[g]);
            int32_t qq[2] = {q0[g], q1[g]};
            cplx ks[2][16];
            memset(ks, 0, sizeof ks);
            if (noisy && noise[g] == N_PHASE) {
                double P = exp(-e * e);
                /* U_theta E1 = diag(1, 1, 1, e^{-i theta} sqrt P), U_theta E2 = diag(0, 0, 0, e^{-i theta} sqrt(1-P)) */
                ks[0][0] = 1; ks[0][5] = 1; ks[0][10] = 1; ks[0][15] = ph * sqrt(P);
                ks[1][15] = ph * sqrt(1.0 - P);
                ops_to_doubles(&ks[0][0], 32, buf);
                st = or_dm_apply_kraus(n, rho_out, 2, qq, 2, buf);
            } else {
                ks[0][0] = 1; ks[0][5] = 1; ks[0][10] = 1; ks[0][15] = ph;
                ops_to_doubles(&ks[0][0], 16, buf);
                st = or_dm_apply_kraus(n, rho_out, 2, qq, 1, buf);
            }
            break;
        }
        case K_SWAP:
        case K_CNOT:
        case K_U2: {
            cplx u[16];
            memset(u, 0, sizeof u);
            if (kind[g] == K_SWAP) {
                u[0] = 1; u[4 * 1 + 2] = 1; u[4 * 2 + 1] = 1; u[15] = 1;
            } else if (kind[g] == K_CNOT) {
                /* control q0 (local bit 0), target q1 (local bit 1): |1,t> -> |1,1-t> */
                u[0] = 1; u[4 * 1 + 3] = 1; u[4 * 2 + 2] = 1; u[4 * 3 + 1] = 1;
            } else {
                for (int i = 0; i < 16; ++i)
                    u[i] = m[2 * i] + I * m[2 * i + 1];
            }
            int32_t qq[2] = {q0[g], q1[g]};
            ops_to_doubles(u, 16, buf);
            st = or_dm_apply_kraus(n, rho_out, 2, qq, 1, buf);
            break;
        }
        case K_FLIP: {
            /* F rho F with F = I - 2 sum_{i & mask == value} |i><i|: entry (i, j) changes sign
               when exactly one of row i and column j is selected. */
            for (uint64_t i = 0; i < N; ++i)
                for (uint64_t j = 0; j < N; ++j) {
                    int ri = (i & mask[g]) == value[g];
                    int cj = (j & mask[g]) == value[g];
                    if (ri != cj)
                        rho[i * N + j] = -rho[i * N + j];
                }
            break;
        }
        case K_DIAG: {
            /* D rho D^dagger: entry (i, j) times f when row i is selected, times conj(f) when
               column j is. */
            cplx f = m[0] + I * m[1];
            for (uint64_t i = 0; i < N; ++i)
                for (uint64_t j = 0; j < N; ++j) {
                    if ((i & mask[g]) == value[g])
                        rho[i * N + j] *= f;
                    if ((j & mask[g]) == value[g])
                        rho[i * N + j] *= conj(f);
                }
            break;
        }
        default:
            break;
        }
        if (st != 0)
            return st;
    }
    return 0;
}

/* <psi|rho|psi> = sum_ij conj(psi_i) rho_ij psi_j and Tr rho = sum_i rho_ii. */
void or_dm_expect(int n, const double *rho, const double *psi, double *f_re, double *f_im,
                  double *tr_re, double *tr_im)
{
    uint64_t N = 1ull << n;
    const cplx *r = (const cplx *)rho, *p = (const cplx *)psi;
    cplx f = 0, t = 0;
    for (uint64_t i = 0; i < N; ++i) {
        t += r[i * N + i];
        for (uint64_t j = 0; j < N; ++j)
            f += conj(p[i]) * r[i * N + j] * p[j];
    }
    *f_re = creal(f);
    *f_im = cimag(f);
    *tr_re = creal(t);
    *tr_im = cimag(t);
}
