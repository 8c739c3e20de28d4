// C ABI of libqsim: argument validation, buffer layout, launch orchestration, kernel timing,
// and the host side of the fixed-rank step (FP64 Jacobi eigen-decomposition).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <memory>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace qs {

// ---------------------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------------------
static thread_local std::string g_err;

qs_status fail(qs_status st, const std::string &msg)
{
    g_err = msg;
    return st;
}

qs_status hip_fail(hipError_t e, const char *what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return QS_EDEVICE;
}

void clear_error() { g_err.clear(); }

// ---------------------------------------------------------------------------------------
// Timing
// ---------------------------------------------------------------------------------------
struct TimingRecord {
    const char *name;
    double bytes;
    hipEvent_t a, b;
};

static std::mutex g_tmu;
static std::atomic<bool> g_timing{false};
static std::vector<TimingRecord> g_pending;
struct Acc {
    int64_t n = 0;
    double ms = 0, bytes = 0;
};
static std::vector<std::pair<std::string, Acc>> g_acc;

TimedLaunch::TimedLaunch(const char *nm, double bytes, hipStream_t s) : name(nm), alg_bytes(bytes), st(s)
{
    if (!g_timing) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;   // graphs: untimed
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return;
    if (hipEventRecord(a, st) != hipSuccess) return;
    on = true;
}

TimedLaunch::~TimedLaunch()
{
    if (!on) return;
    (void)hipEventRecord(b, st);
    std::lock_guard<std::mutex> lk(g_tmu);
    g_pending.push_back({name, alg_bytes, a, b});
}

static void timing_flush()
{
    std::lock_guard<std::mutex> lk(g_tmu);
    for (auto &r : g_pending) {
        (void)hipEventSynchronize(r.b);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, r.a, r.b);
        auto it = std::find_if(g_acc.begin(), g_acc.end(), [&](auto &p) { return p.first == r.name; });
        if (it == g_acc.end()) {
            g_acc.push_back({r.name, Acc()});
            it = g_acc.end() - 1;
        }
        it->second.n += 1;
        it->second.ms += ms;
        it->second.bytes += r.bytes;
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_pending.clear();
}

}  // namespace qs

using namespace qs;

// ---------------------------------------------------------------------------------------
// Handles
// ---------------------------------------------------------------------------------------
struct qs_state_s {
    int n;
    qs_dtype dt;
    int T;
    void *buf;
    size_t bytes;
    hipStream_t st;
    double *scratch;     // device: table rows, reduction partials, outputs, and (last 512
                         // doubles) the superoperator of a two-qubit Kraus set
    size_t scratch_doubles;
    double *kraus_host = nullptr;     // pinned staging of that superoperator (first use)
    hipEvent_t kraus_ev = nullptr;    // its last upload (the staging is reused after it)
};

struct qs_fr_s {
    int n, r, rank;
    qs_dtype dt;
    void *V;
    hipStream_t st;
    double log_trace;
    double *scratch;     // device: gram partials | gram out | coef | overlap partials | out | table
    size_t off_gram, off_coef, off_ovp, off_ovo, off_tab;
    double *host;        // pinned staging: gram, then coef (kFrHostGram doubles each)
};

// Doubles of one Gram or coefficient matrix: 32 x 32 complex (two-qubit Kraus sets; a
// one-qubit set uses the leading 16 x 16).
constexpr size_t kFrHostGram = 32 * 32 * 2;

static size_t state_bytes(int n, qs_dtype dt, int T) { return ((size_t)T << n) * amp_bytes(dt); }


extern "C" {

const char *qs_last_error(void) { return g_err.c_str(); }
const char *qs_version(void) { return "qsim-gfx950 1.0"; }

size_t qs_sv_bytes_required(int n, qs_dtype dt, int T)
{
    if (n < 1 || n > 34 || T < 1 || (dt != QS_C64 && dt != QS_C128)) return 0;
    return state_bytes(n, dt, T);
}

qs_status qs_sv_create(int n, qs_dtype dt, int T, void *buf, size_t bytes, void *stream, qs_state *out)
{
    clear_error();
    if (!out) return fail(QS_EINVAL, "sv_create: out is NULL");
    *out = nullptr;
    if (n < 1 || n > 34) return fail(QS_EINVAL, "sv_create: n_qubits must be in 1..34");
    if (dt != QS_C64 && dt != QS_C128) return fail(QS_EINVAL, "sv_create: unknown dtype");
    if (T < 1) return fail(QS_EINVAL, "sv_create: n_traj must be >= 1");
    if (!buf || !aligned256(buf)) return fail(QS_EINVAL, "sv_create: buffer must be non-NULL and 256-byte aligned");
    if (bytes < state_bytes(n, dt, T)) return fail(QS_EINVAL, "sv_create: buffer too small");
    auto *s = new (std::nothrow) qs_state_s();
    if (!s) return fail(QS_ENOMEM, "sv_create: out of host memory");
    s->n = n;
    s->dt = dt;
    s->T = T;
    s->buf = buf;
    s->bytes = bytes;
    s->st = (hipStream_t)stream;
    s->scratch_doubles = (size_t)T * 8 + reduce_partials_doubles(n, T) + 2 * reduce_partials_doubles(n, 1) + 64 +
                         (size_t)T * 5 + 64 + 512;
    hipError_t e = hipMalloc(&s->scratch, s->scratch_doubles * sizeof(double));
    if (e != hipSuccess) {
        delete s;
        return hip_fail(e, "sv_create: hipMalloc scratch");
    }
    *out = s;
    return QS_OK;
}

qs_status qs_sv_destroy(qs_state s)
{
    clear_error();
    if (!s) return QS_OK;
    (void)hipStreamSynchronize(s->st);
    (void)hipFree(s->scratch);
    if (s->kraus_ev) (void)hipEventDestroy(s->kraus_ev);
    if (s->kraus_host) (void)hipHostFree(s->kraus_host);
    delete s;
    return QS_OK;
}

qs_status qs_sv_init_basis(qs_state s, uint64_t index)
{
    clear_error();
    if (!s) return fail(QS_EINVAL, "sv_init_basis: NULL state");
    if (index >= (1ull << s->n)) return fail(QS_EINVAL, "sv_init_basis: index out of range");
    QS_HIP(launch_init_basis(s->buf, s->dt, s->n, s->T, index, s->st));
    return QS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------
// Gate validation and the single-gate sweep
// ---------------------------------------------------------------------------------------
static qs_status check_gate(const qs_gate &g, int n, int idx)
{
    auto bad = [&](const char *why) {
        return fail(QS_EINVAL, "gate " + std::to_string(idx) + ": " + why);
    };
    const uint64_t nmask = (n >= 64) ? ~0ull : ((1ull << n) - 1);
    switch (g.kind) {
    case QS_G_U1:
        if (g.q0 < 0 || g.q0 >= n) return bad("qubit out of range");
        if (g.noise != QS_NOISE_NONE && g.noise != QS_NOISE_ROT) return bad("U1 takes no or ROT noise");
        break;
    case QS_G_CP:
    case QS_G_SWAP:
    case QS_G_CNOT:
    case QS_G_U2:
        if (g.q0 < 0 || g.q0 >= n || g.q1 < 0 || g.q1 >= n) return bad("qubit out of range");
        if (g.q0 == g.q1) return bad("two-qubit gate on one qubit");
        if (g.kind == QS_G_CP && g.noise != QS_NOISE_NONE && g.noise != QS_NOISE_PHASE)
            return bad("CP takes no or PHASE noise");
        if (g.kind != QS_G_CP && g.noise != QS_NOISE_NONE) return bad("noise only on U1 and CP");
        break;
    case QS_G_FLIP:
    case QS_G_DIAG:
        if (g.mask & ~nmask) return bad("FLIP/DIAG mask beyond n bits");
        if (g.value & ~g.mask) return bad("FLIP/DIAG value outside its mask");
        if (g.noise != QS_NOISE_NONE) return bad("noise only on U1 and CP");
        break;
    default:
        return bad("unknown gate kind");
    }
    if (!std::isfinite(g.theta)) return bad("non-finite theta");
    for (double v : g.m)
        if (!std::isfinite(v)) return bad("non-finite matrix entry");
    return QS_OK;
}

static qs_status check_noise(const qs_noise *nz, int T)
{
    if (!nz) return QS_OK;
    if (!std::isfinite(nz->e) || nz->e < 0) return fail(QS_EINVAL, "noise: e must be finite and >= 0");
    if (nz->e_per_traj)
        for (int t = 0; t < T; ++t)
            if (!std::isfinite(nz->e_per_traj[t]) || nz->e_per_traj[t] < 0)
                return fail(QS_EINVAL, "noise: e_per_traj entries must be finite and >= 0");
    return QS_OK;
}

static const double kCnot4[32] = {1, 0, 0, 0, 0, 0, 0, 0,  0, 0, 0, 0, 0, 0, 1, 0,
                                  0, 0, 0, 0, 1, 0, 0, 0,  0, 0, 1, 0, 0, 0, 0, 0};

// Apply gate g to S slots of psi; tab_scratch holds S * 8 doubles.
static qs_status sweep_gate(void *psi, qs_dtype dt, int n, int S, const qs_gate &g,
                            const qs_noise *nz, double *tab_scratch, hipStream_t st)
{
    if (g.kind == QS_G_U1 || g.kind == QS_G_CP) {
        NoiseArgs na{};
        na.e = nz ? nz->e : 0.0;
        na.e_dev = nullptr;
        na.seed = nz ? nz->seed : 0;
        na.request = nz ? nz->request : 0;
        na.traj_base = nz ? nz->traj_base : 0;
        na.first_noisy_slot = 0;
        QS_HIP(launch_noise_one(g, S, na, tab_scratch, st));
        if (g.kind == QS_G_U1) QS_HIP(launch_sweep_u1(psi, dt, n, S, g.q0, tab_scratch, st));
        else QS_HIP(launch_sweep_cp(psi, dt, n, S, g.q0, g.q1, tab_scratch, st));
    } else if (g.kind == QS_G_SWAP || g.kind == QS_G_CNOT) {
        QS_HIP(launch_sweep_perm(psi, dt, n, S, g.kind, g.q0, g.q1, st));
    } else if (g.kind == QS_G_U2) {
        QS_HIP(launch_sweep_2q(psi, dt, n, S, g.q0, g.q1, g.m, st));
    } else if (g.kind == QS_G_FLIP) {
        QS_HIP(launch_flip(psi, dt, n, S, g.mask, g.value, st));
    } else if (g.kind == QS_G_DIAG) {
        QS_HIP(launch_scale_pattern(psi, dt, n, S, g.mask, g.value, g.m[0], g.m[1], st));
    }
    return QS_OK;
}

// Kraus set of the eq. (1) noisy one-qubit gate U: {U E1, U E2}, E1 = sqrt(l1) I,
// E2 = sqrt(l2) [[0, 1], [-1, 0]], l1,2 = (1 +- exp(-2 e^2)) / 2 (eq. 6).  out: 2 x 8 doubles.
static void kraus_rot_ops(const double *u, double e, double *out)
{
    const double l1 = 0.5 * (1.0 + std::exp(-2.0 * e * e));
    const double l2 = 0.5 * (1.0 - std::exp(-2.0 * e * e));
    const double s1 = std::sqrt(l1), s2 = std::sqrt(l2);
    for (int r = 0; r < 2; ++r) {
        std::complex<double> a(u[4 * r], u[4 * r + 1]), b(u[4 * r + 2], u[4 * r + 3]);
        std::complex<double> k1c0 = a * s1, k1c1 = b * s1;      // U E1
        std::complex<double> k2c0 = -b * s2, k2c1 = a * s2;     // U E2: columns (-U_r1, U_r0) sqrt(l2)
        out[4 * r] = k1c0.real(); out[4 * r + 1] = k1c0.imag();
        out[4 * r + 2] = k1c1.real(); out[4 * r + 3] = k1c1.imag();
        out[8 + 4 * r] = k2c0.real(); out[8 + 4 * r + 1] = k2c0.imag();
        out[8 + 4 * r + 2] = k2c1.real(); out[8 + 4 * r + 3] = k2c1.imag();
    }
}

extern "C" {

qs_status qs_apply_gate(qs_state s, const qs_gate *g, const qs_noise *nz)
{
    clear_error();
    if (!s || !g) return fail(QS_EINVAL, "apply_gate: NULL argument");
    qs_status v = check_gate(*g, s->n, 0);
    if (v != QS_OK) return v;
    if ((v = check_noise(nz, s->T)) != QS_OK) return v;
    if (nz && nz->e_per_traj) return fail(QS_EUNSUPPORTED, "apply_gate: e_per_traj is for run_trajectories");
    return sweep_gate(s->buf, s->dt, s->n, s->T, *g, nz, s->scratch, s->st);
}

}  // extern "C"

// Two-qubit Kraus set on vec(rho): S = sum_o E_o (x) conj(E_o) on the four index bits
// (bra q0, bra q1, ket q0 + n, ket q1 + n), local index l = b + 4 a for the ket local index
// a = bit(q0 + n) + 2 bit(q1 + n) and the bra local index b = bit(q0) + 2 bit(q1):
// S[(a, b), (c, d)] = sum_o E_o[a][c] conj(E_o[b][d]) (eq. 3; operators row-major on the local
// index bit(q0) + 2 bit(q1)).  Built in FP64 on the host, staged through pinned memory.
static qs_status apply_kraus2(qs_state rho, int n, const int32_t *q, int n_ops, const double *ops)
{
    if (!rho->kraus_host) {
        QS_HIP(hipHostMalloc((void **)&rho->kraus_host, 512 * sizeof(double), hipHostMallocDefault));
        QS_HIP(hipEventCreateWithFlags(&rho->kraus_ev, hipEventDisableTiming));
    } else {
        QS_HIP(hipEventSynchronize(rho->kraus_ev));   // the previous upload has read the staging
    }
    double *S = rho->kraus_host;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b)
            for (int c = 0; c < 4; ++c)
                for (int d = 0; d < 4; ++d) {
                    std::complex<double> v = 0;
                    for (int o = 0; o < n_ops; ++o) {
                        const double *E = ops + 32 * o;
                        std::complex<double> eac(E[2 * (4 * a + c)], E[2 * (4 * a + c) + 1]);
                        std::complex<double> ebd(E[2 * (4 * b + d)], E[2 * (4 * b + d) + 1]);
                        v += eac * std::conj(ebd);
                    }
                    const int row = b + 4 * a, col = d + 4 * c;
                    S[2 * (16 * row + col)] = v.real();
                    S[2 * (16 * row + col) + 1] = v.imag();
                }
    double *m_dev = rho->scratch + rho->scratch_doubles - 512;
    QS_HIP(hipMemcpyAsync(m_dev, S, 512 * sizeof(double), hipMemcpyHostToDevice, rho->st));
    QS_HIP(hipEventRecord(rho->kraus_ev, rho->st));
    const int bits[4] = {q[0], q[1], q[0] + n, q[1] + n};
    QS_HIP(launch_sweep_4q(rho->buf, rho->dt, rho->n, bits, m_dev, rho->st));
    return QS_OK;
}

extern "C" {

qs_status qs_apply_kraus(qs_state rho, int k, const int32_t *qubits, int n_ops, const double *ops)
{
    clear_error();
    if (!rho || !qubits || !ops) return fail(QS_EINVAL, "apply_kraus: NULL argument");
    if (rho->n % 2 != 0) return fail(QS_EINVAL, "apply_kraus: state must have 2n qubits (vec rho)");
    if (rho->T != 1) return fail(QS_EINVAL, "apply_kraus: density matrix state must hold one vector");
    const int n = rho->n / 2;
    if (k != 1 && k != 2) return fail(QS_EUNSUPPORTED, "apply_kraus: one- and two-qubit Kraus sets (k = 1, 2) only");
    for (int i = 0; i < k; ++i)
        if (qubits[i] < 0 || qubits[i] >= n) return fail(QS_EINVAL, "apply_kraus: qubit out of range");
    if (k == 2 && qubits[0] == qubits[1]) return fail(QS_EINVAL, "apply_kraus: the two qubits must differ");
    if (n_ops < 1 || n_ops > 64) return fail(QS_EINVAL, "apply_kraus: n_ops must be in 1..64");
    const int dim = 1 << k;
    for (int i = 0; i < n_ops * dim * dim * 2; ++i)
        if (!std::isfinite(ops[i])) return fail(QS_EINVAL, "apply_kraus: non-finite operator entry");
    if (k == 2) return apply_kraus2(rho, n, qubits, n_ops, ops);
    // Superoperator S = sum_k E_k (x) conj(E_k) on (bra bit q, ket bit q + n): local index
    // bit(q) + 2 bit(q + n) = b + 2 a for ket bit a, bra bit b;
    // S[(a, b), (c, d)] = sum_k E_k[a][c] conj(E_k[b][d]).
    qs_gate g{};
    g.kind = QS_G_U2;
    g.q0 = qubits[0];
    g.q1 = qubits[0] + n;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 2; ++c)
                for (int d = 0; d < 2; ++d) {
                    std::complex<double> s = 0;
                    for (int o = 0; o < n_ops; ++o) {
                        const double *E = ops + 8 * o;
                        std::complex<double> eac(E[2 * (2 * a + c)], E[2 * (2 * a + c) + 1]);
                        std::complex<double> ebd(E[2 * (2 * b + d)], E[2 * (2 * b + d) + 1]);
                        s += eac * std::conj(ebd);
                    }
                    int row = b + 2 * a, col = d + 2 * c;
                    g.m[2 * (4 * row + col)] = s.real();
                    g.m[2 * (4 * row + col) + 1] = s.imag();
                }
    return sweep_gate(rho->buf, rho->dt, rho->n, 1, g, nullptr, rho->scratch, rho->st);
}

qs_status qs_dm_apply_gate(qs_state rho, const qs_gate *g, double e)
{
    clear_error();
    if (!rho || !g) return fail(QS_EINVAL, "dm_apply_gate: NULL argument");
    if (rho->n % 2 != 0 || rho->T != 1) return fail(QS_EINVAL, "dm_apply_gate: rho must be one vector of 2n qubits");
    if (!std::isfinite(e) || e < 0) return fail(QS_EINVAL, "dm_apply_gate: e must be finite and >= 0");
    const int n = rho->n / 2;
    qs_status v = check_gate(*g, n, 0);
    if (v != QS_OK) return v;
    if (g->kind == QS_G_U1) {
        double ops[16];
        int nops = 1;
        if (e > 0 && g->noise == QS_NOISE_ROT) {
            kraus_rot_ops(g->m, e, ops);
            nops = 2;
        } else {
            std::memcpy(ops, g->m, 8 * sizeof(double));
        }
        int32_t q = g->q0;
        return qs_apply_kraus(rho, 1, &q, nops, ops);
    }
    if (g->kind == QS_G_FLIP) {
        QS_HIP(launch_flip(rho->buf, rho->dt, rho->n, 1, g->mask << n, g->value << n, rho->st));
        QS_HIP(launch_flip(rho->buf, rho->dt, rho->n, 1, g->mask, g->value, rho->st));
        return QS_OK;
    }
    if (g->kind == QS_G_DIAG) {
        // the factor on the selected rows, its conjugate on the selected columns
        QS_HIP(launch_scale_pattern(rho->buf, rho->dt, rho->n, 1, g->mask << n, g->value << n, g->m[0], g->m[1],
                                    rho->st));
        QS_HIP(launch_scale_pattern(rho->buf, rho->dt, rho->n, 1, g->mask, g->value, g->m[0], -g->m[1], rho->st));
        return QS_OK;
    }
    if (g->kind == QS_G_CP && e > 0 && g->noise == QS_NOISE_PHASE) {
        // The average over xi of U(theta + e xi) rho U(theta + e xi)^dagger (the channel of
        // eq. 9): rho_ij gets exp(-i theta (b_i - b_j)) exp(-e^2 (b_i - b_j)^2 / 2), b = 1 when
        // both qubits are 1.  Three pattern sweeps: rows with b_i = 1 by f = exp(-i theta) sqrt(P),
        // columns with b_j = 1 by conj(f), and entries with both by 1 / P (P = exp(-e^2)).
        const uint64_t cm = (1ull << g->q0) | (1ull << g->q1);
        const double P = std::exp(-e * e), sp = std::exp(-0.5 * e * e);
        const double fre = std::cos(g->theta) * sp, fim = -std::sin(g->theta) * sp;
        QS_HIP(launch_scale_pattern(rho->buf, rho->dt, rho->n, 1, cm << n, cm << n, fre, fim, rho->st));
        QS_HIP(launch_scale_pattern(rho->buf, rho->dt, rho->n, 1, cm, cm, fre, -fim, rho->st));
        QS_HIP(launch_scale_pattern(rho->buf, rho->dt, rho->n, 1, cm | (cm << n), cm | (cm << n), 1.0 / P, 0.0,
                                    rho->st));
        return QS_OK;
    }
    // two-qubit unitary: U on the ket bits, conj(U) on the bra bits
    qs_gate ket = *g, bra = *g;
    ket.q0 += n;
    ket.q1 += n;
    ket.noise = bra.noise = QS_NOISE_NONE;
    if (g->kind == QS_G_CP) bra.theta = -g->theta;
    if (g->kind == QS_G_U2)
        for (int k = 0; k < 16; ++k) bra.m[2 * k + 1] = -g->m[2 * k + 1];
    v = sweep_gate(rho->buf, rho->dt, rho->n, 1, ket, nullptr, rho->scratch, rho->st);
    if (v != QS_OK) return v;
    return sweep_gate(rho->buf, rho->dt, rho->n, 1, bra, nullptr, rho->scratch + 8, rho->st);
}

qs_status qs_fidelity(qs_state a, int ta, qs_state b, int tb, double *f, double *overlap)
{
    clear_error();
    if (!a || !b || !f) return fail(QS_EINVAL, "fidelity: NULL argument");
    if (a->n != b->n || a->dt != b->dt) return fail(QS_EINVAL, "fidelity: states differ in n or dtype");
    if (ta < 0 || ta >= a->T || tb < 0 || tb >= b->T) return fail(QS_EINVAL, "fidelity: trajectory out of range");
    const int n = a->n;
    const size_t sb = amp_bytes(a->dt) << n;
    double *part = a->scratch + (size_t)a->T * 8;
    double *out = a->scratch + a->scratch_doubles - 64 - 16;
    const char *pa = (const char *)a->buf + sb * ta;
    const char *pb = (const char *)b->buf + sb * tb;
    if (a->st != b->st) QS_HIP(hipStreamSynchronize(b->st));
    QS_HIP(launch_overlaps(pa, 0, pb, a->dt, n, 1, -1, part, out, a->st));
    QS_HIP(launch_overlaps(pa, 0, pa, a->dt, n, 1, -1, part, out + 5, a->st));
    double h[10];
    QS_HIP(hipMemcpyAsync(h, out, sizeof h, hipMemcpyDeviceToHost, a->st));
    QS_HIP(hipStreamSynchronize(a->st));
    double nb = h[2], na = h[7];
    *f = (h[0] * h[0] + h[1] * h[1]) / (na * nb);
    if (overlap) {
        overlap[0] = h[0];
        overlap[1] = h[1];
    }
    return QS_OK;
}

qs_status qs_dm_fidelity(qs_state rho, qs_state psi, int tpsi, double *f, double *trace)
{
    clear_error();
    if (!rho || !psi || !f) return fail(QS_EINVAL, "dm_fidelity: NULL argument");
    if (rho->T != 1 || rho->n != 2 * psi->n || rho->dt != psi->dt)
        return fail(QS_EINVAL, "dm_fidelity: rho must be one vector of 2n qubits with psi's dtype");
    if (tpsi < 0 || tpsi >= psi->T) return fail(QS_EINVAL, "dm_fidelity: trajectory out of range");
    const int n = psi->n;
    const char *pp = (const char *)psi->buf + (amp_bytes(psi->dt) << n) * tpsi;
    double *part = rho->scratch + 8;
    double *out = rho->scratch + rho->scratch_doubles - 64 - 16;
    if (rho->st != psi->st) QS_HIP(hipStreamSynchronize(psi->st));
    QS_HIP(launch_dm_expect(rho->buf, pp, rho->dt, n, part, out, rho->st));
    double h[4];
    QS_HIP(hipMemcpyAsync(h, out, sizeof h, hipMemcpyDeviceToHost, rho->st));
    QS_HIP(hipStreamSynchronize(rho->st));
    *f = h[0];
    if (trace) *trace = h[2];
    return QS_OK;
}

qs_status qs_noise_draw(uint64_t seed, uint32_t request, uint32_t stream, const uint32_t *sites_dev,
                        int n_sites, uint32_t traj_base, int n_traj, double *out_dev, void *hip_stream)
{
    clear_error();
    if (!sites_dev || !out_dev) return fail(QS_EINVAL, "noise_draw: NULL argument");
    if (n_sites < 0 || n_traj < 0) return fail(QS_EINVAL, "noise_draw: negative size");
    QS_HIP(launch_noise_draw(seed, request, stream, sites_dev, n_sites, traj_base, n_traj, out_dev,
                             (hipStream_t)hip_stream));
    return QS_OK;
}

qs_status qs_copy(void *dst, const void *src, size_t bytes, void *hip_stream)
{
    clear_error();
    if (!dst || !src || bytes % 16) return fail(QS_EINVAL, "copy: NULL pointer or size not a multiple of 16");
    QS_HIP(launch_copy(dst, src, bytes, (hipStream_t)hip_stream));
    return QS_OK;
}

qs_status qs_timing_enable(int on)
{
    clear_error();
    timing_flush();
    g_timing = on != 0;
    return QS_OK;
}

qs_status qs_timing_read(const char *name, int64_t *launches, double *ms, double *alg_bytes)
{
    clear_error();
    if (!name) return fail(QS_EINVAL, "timing_read: NULL name");
    timing_flush();
    std::lock_guard<std::mutex> lk(g_tmu);
    for (auto &p : g_acc)
        if (p.first == name) {
            if (launches) *launches = p.second.n;
            if (ms) *ms = p.second.ms;
            if (alg_bytes) *alg_bytes = p.second.bytes;
            return QS_OK;
        }
    if (launches) *launches = 0;
    if (ms) *ms = 0;
    if (alg_bytes) *alg_bytes = 0;
    return QS_OK;
}

qs_status qs_timing_reset(void)
{
    clear_error();
    timing_flush();
    std::lock_guard<std::mutex> lk(g_tmu);
    g_acc.clear();
    return QS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------
// run_trajectories
// ---------------------------------------------------------------------------------------
namespace {

struct TrajLayout {
    size_t states, tab, gates, edev, passes, stages, rounds, ops, prefs, jobs, obits, chains, wtab, rec, partials, out,
        dyn, total;
};

struct Plan {
    bool fused = false;
    bool mfma = false;
    int K = 0, RB = 0, run_bits = 0;
    qs::Program prog;
};

qs_status fused_plan_for(const qs_gate *gates, int n_gates, int n, qs_dtype dt, int K, int RB, int run,
                         Plan &out, bool mfma = false)
{
    out.fused = true;
    if (K > kMaxTileBits) return fail(QS_EINVAL, "plan: tile_bits too large");
    if ((size_t(1) << std::min(K, n)) * amp_bytes(dt) > 160 * 1024)
        return fail(QS_EINVAL, "plan: tile does not fit the 160 KiB LDS of a gfx950 CU");
    if (RB > kMaxRegBits) return fail(QS_EINVAL, "plan: reg_bits must be <= 4");
    if (n <= K) {
        K = n;   // the whole state is one tile: the circuit runs as one launch
        if (RB > K) RB = K;
    }
    // wide register tiles (16 complex<float>, 8 or 16 complex<double>) run 256-thread blocks
    if ((RB == 4 || (dt == QS_C128 && RB == 3)) && K - RB > 8)
        return fail(QS_EINVAL, "plan: this register tile allows at most 256 threads (tile_bits - reg_bits <= 8)");
    out.K = K;
    out.RB = RB;
    out.run_bits = run;
    int rec_cap = stage_rec_cap(dt, K);
    if (rec_cap < 256) return fail(QS_EINVAL, "plan: tile leaves too little LDS for the gate records");
    out.mfma = mfma && dt == QS_C64 && RB == 4;
    return plan_fused(gates, n_gates, n, K, RB, run, rec_cap, out.prog, out.mfma);
}

// ---------------------------------------------------------------------------------------
// Plan cost model: seconds per state slot.  Each fused pass costs the larger of its HBM time
// (one read and one write of the state, the first pass only a write) and its vector-ALU time
// (per-amplitude instruction counts of each op kind, measured from the kernel's code), plus
// the launch of its prep and pass kernels; an unfused run costs each gate's sweep.  The
// constants are properties of the kernels on gfx950, so the choice is a pure function of the
// circuit, n and the dtype.
// ---------------------------------------------------------------------------------------
constexpr double kModelHbm = 5.5e12;          // sustained bytes/s of a streaming kernel
constexpr double kModelValu = 39.3e12 * 0.9;  // lane-instructions/s: 1024 SIMDs x 64 lanes / 4 cycles
                                              // x 2.4 GHz, at the utilisation the pass reaches
constexpr double kModelLaunch = 8e-6;         // s per pass (two launches, amortised over slots below)
constexpr int kModelSlots = 64;

// Fraction of the streaming bandwidth reached with rows of 2^run_bits contiguous amplitudes
// (measured with the fused pass: rows of 128 bytes stream as well as longer ones).
static double row_efficiency(int run_bits, qs_dtype dt)
{
    const double bytes = std::ldexp((double)amp_bytes(dt), run_bits);
    return bytes >= 128 ? 1.0 : bytes >= 64 ? 0.8 : bytes >= 32 ? 0.45 : 0.3;
}

// A dense 16 x 16 block on the FP32 matrix cores: 64 products of 16 x 16 x 4 per 1024 amplitudes
// (one wave's tile), 32 cycles each on one SIMD's matrix unit: 2 cycles per amplitude, the
// vector-ALU equivalent of 2 x 16 lane-instructions per amplitude at the model's issue rate.
constexpr double kModelBlockValuEq = 32.0;

double model_cost_fused(const Program &P, int n, qs_dtype dt, int S, int run_bits)
{
    const double N = std::ldexp(1.0, n), amp = (double)amp_bytes(dt);
    const double wide = dt == QS_C128 ? 2.0 : 1.0;   // FP64 arithmetic: twice the instructions
    const double eff = P.passes.size() && P.passes[0].outer_mask ? row_efficiency(run_bits, dt) : 1.0;
    double total = 0.0;
    for (size_t pi = 0; pi < P.passes.size(); ++pi) {
        const PassDesc &pd = P.passes[pi];
        double per_amp = 20.0;                                  // load/store, tile set-up
        per_amp += 6.0 * (pd.round_end - pd.round_begin + 1);   // LDS exchanges
        if (pd.blocks) {
            // block rounds: the matrix-core time, the lane exchanges around each block (4 per
            // amplitude) and the phases applied outside the block (5 per folded block)
            for (int ri = pd.round_begin; ri < pd.round_end; ++ri) {
                per_amp += kModelBlockValuEq + 4.0;
                for (int oi = P.rounds[ri].op_begin; oi < P.rounds[ri].op_end; ++oi) {
                    const OpDesc &op = P.ops[oi];
                    per_amp += 5.0 * ((op.pre_rec >= 0) + (op.post_rec >= 0));
                }
            }
            const double mem = (pi == 0 ? 1.0 : 2.0) * N * amp / (kModelHbm * eff);
            const double alu = N * per_amp / kModelValu;
            total += std::max(mem, alu) + 0.5 * std::min(mem, alu);
            continue;
        }
        for (int oi = pd.op_begin; oi < pd.op_end; ++oi) {
            const OpDesc &op = P.ops[oi];
            if (op.type == OP_U1) {
                per_amp += (op.flags & OPF_REAL) ? 7.0 : 10.0;
                per_amp += 5.0 * ((op.pre_rec >= 0) + (op.post_rec >= 0));
            } else if (op.type == OP_U2) {
                per_amp += 27.0;
            } else {
                per_amp += 5.0;
            }
        }
        const double mem = (pi == 0 ? 1.0 : 2.0) * N * amp / (kModelHbm * eff);
        const double alu = N * per_amp * wide / kModelValu;
        // the two overlap only in part: a pass waits on both its loads and its arithmetic
        double pass = std::max(mem, alu) + 0.5 * std::min(mem, alu);
        if (dt == QS_C128 && pd.zin_ops == 5) {
            // a pass without one-qubit ops holds few registers, so its occupancy is set by the
            // LDS its tile takes: a 64 KiB tile leaves two waves per SIMD, which measured 10 %
            // slower than smaller tiles at four or more (density-matrix superoperator passes)
            const int blocks = (int)((160u * 1024u) / ((size_t(1) << pd.K) * 16u));
            const int waves = blocks * (1 << (pd.K - pd.RB)) / 64 / 4;
            if (waves < 4) pass /= waves <= 2 ? 0.85 : 0.92;
        }
        total += pass;
    }
    return total + kModelLaunch * (double)P.passes.size() / std::max(S, 1);
}

double model_cost_unfused(const qs_gate *gates, int n_gates, int n, qs_dtype dt, int S)
{
    const double N = std::ldexp(1.0, n), amp = (double)amp_bytes(dt);
    double t = N * amp / kModelHbm;   // initial state
    for (int g = 0; g < n_gates; ++g) {
        double frac = 1.0;
        switch (gates[g].kind) {
        case QS_G_CP: frac = 0.5; break;   // touches N/4 amplitudes in lines of half the state
        case QS_G_SWAP: frac = 1.0; break;
        case QS_G_FLIP:
        case QS_G_DIAG: frac = 0.0; break;
        default: frac = 1.0;
        }
        t += 2.0 * frac * N * amp / kModelHbm + 4e-6 / std::max(S, 1);
    }
    return t;
}

// Candidate shapes per dtype: (tile bits, register bits, run bits).
static const int kCandC64[][3] = {{12, 4, 4}, {12, 4, 5}, {12, 3, 5}, {12, 3, 4}, {12, 3, 3}, {11, 3, 4},
                                  {11, 2, 3}, {10, 2, 3}};
static const int kCandC128[][3] = {{11, 3, 4}, {11, 3, 3}, {11, 2, 4}, {11, 2, 3}, {10, 2, 3}, {10, 1, 3},
                                   {12, 4, 3}, {12, 4, 4}};

qs_status autotune_plan(const qs_gate *gates, int n_gates, int n, qs_dtype dt, int S, Plan &out,
                        double *cost_out)
{
    bool two_qubit_dense = false;
    for (int g = 0; g < n_gates; ++g)
        if (gates[g].kind == QS_G_U2 || gates[g].kind == QS_G_CNOT) two_qubit_dense = true;
    double best = model_cost_unfused(gates, n_gates, n, dt, S);
    out = Plan();
    out.fused = false;
    const int ncand = dt == QS_C64 ? (int)(sizeof kCandC64 / sizeof kCandC64[0])
                                   : (int)(sizeof kCandC128 / sizeof kCandC128[0]);
    for (int c = 0; c < ncand; ++c) {
        const int *k = dt == QS_C64 ? kCandC64[c] : kCandC128[c];
        if (two_qubit_dense && k[1] < 2) continue;
        // complex<float> shapes with 16 registers also as block-round plans (matrix cores)
        for (int mf = 0; mf <= (dt == QS_C64 && k[1] == 4 ? 1 : 0); ++mf) {
            Plan cand;
            if (fused_plan_for(gates, n_gates, n, dt, k[0], k[1], k[2], cand, mf == 1) != QS_OK) {
                clear_error();
                continue;
            }
            const double cost = model_cost_fused(cand.prog, n, dt, S, cand.run_bits);
            if (cost < best * 0.999) {
                best = cost;
                out = std::move(cand);
            }
        }
    }
    if (cost_out) *cost_out = best;
    return QS_OK;
}

qs_status resolve_plan(const qs_gate *gates, int n_gates, int n, qs_dtype dt, int T, const qs_plan *p,
                       Plan &out)
{
    int fuse = p ? p->fuse : -1;
    if (fuse < -1 || fuse > 1) return fail(QS_EINVAL, "plan: fuse must be -1, 0 or 1");
    const bool shape_given = p && (p->tile_bits > 0 || p->reg_bits > 0 || p->run_bits > 0);
    // the automatic choice is priced for a batch of 64 slots whatever T is, so that every batch
    // of a request (and the request alone) gets the same plan
    (void)T;
    if (fuse == -1 && !shape_given) return autotune_plan(gates, n_gates, n, dt, kModelSlots, out, nullptr);
    if (fuse == -1) fuse = 1;
    out.fused = fuse == 1;
    if (!out.fused) return QS_OK;
    // defaults: 2^12-amplitude tiles of 16 registers per thread over 256 threads, the largest
    // register tiles that stay out of scratch memory (complex<double> at two waves per SIMD);
    // rows of 16 amplitudes (128 B, 256 B), the fastest measured
    int K = (p && p->tile_bits > 0) ? p->tile_bits : 12;
    int RB = (p && p->reg_bits > 0) ? p->reg_bits : 4;
    int run = (p && p->run_bits > 0) ? p->run_bits : 4;
    if (p && (p->mfma < 0 || p->mfma > 1)) return fail(QS_EINVAL, "plan: mfma must be 0 or 1");
    return fused_plan_for(gates, n_gates, n, dt, K, RB, run, out, p && p->mfma == 1);
}

TrajLayout traj_layout(int n, qs_dtype dt, int T, int n_gates, const Plan &pl)
{
    TrajLayout L{};
    const int S = T + 1;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align256(off + bytes);
        return at;
    };
    L.states = take(state_bytes(n, dt, S));
    L.tab = take((size_t)n_gates * S * 8 * sizeof(double));
    L.gates = take((size_t)std::max(n_gates, 1) * sizeof(qs_gate));
    L.edev = take((size_t)S * sizeof(double));
    L.passes = take(std::max<size_t>(pl.prog.passes.size(), 1) * sizeof(PassDesc));
    L.stages = take(std::max<size_t>(pl.prog.stages.size(), 1) * sizeof(StageDesc));
    L.rounds = take(std::max<size_t>(pl.prog.rounds.size(), 1) * sizeof(RoundDesc));
    L.ops = take(std::max<size_t>(pl.prog.ops.size(), 1) * sizeof(OpDesc));
    L.prefs = take(std::max<size_t>(pl.prog.prefs.size(), 1) * sizeof(PrepRef));
    L.jobs = take(std::max<size_t>(pl.prog.jobs.size(), 1) * sizeof(OuterJob));
    L.obits = take(std::max<size_t>(pl.prog.obits.size(), 1) * sizeof(int32_t));
    L.chains = take(std::max<size_t>(pl.prog.chain_gates.size() + pl.prog.chain_off.size(), 1) * sizeof(int32_t));
    // the tiles' outer index bits (at most 2^(n - K) tiles), then the per (slot, tile, outer job)
    // phase products of the pass being run
    {
        const int tb = pl.fused && n > pl.prog.K ? n - pl.prog.K : 0;
        const size_t entries = ((size_t)S << tb) * (size_t)std::max(pl.prog.max_jobs, 1);
        L.wtab = take(align256((size_t(1) << tb) * sizeof(uint64_t)) + entries * 2 * (dt == QS_C64 ? 4 : 8));
    }
    L.rec = take((size_t)std::max(pl.prog.max_rec, 1) * S * 2 * (dt == QS_C64 ? 4 : 8));
    {
        // the fused runs' per (slot, tile) overlap partials of their last pass
        size_t d = reduce_partials_doubles(n, S);
        if (pl.fused) {
            const int tb = n > pl.prog.K ? n - pl.prog.K : 0;
            d = std::max(d, ((size_t)S << tb) * 3);
        }
        L.partials = take(d * sizeof(double));
    }
    L.out = take((size_t)S * 5 * sizeof(double));
    L.dyn = take(sizeof(RunParams));
    L.total = off;
    return L;
}

qs_status check_circuit(const qs_gate *gates, int n_gates, int n)
{
    if (n_gates < 0) return fail(QS_EINVAL, "n_gates must be >= 0");
    if (n_gates > 0 && !gates) return fail(QS_EINVAL, "gates is NULL");
    for (int i = 0; i < n_gates; ++i) {
        qs_status v = check_gate(gates[i], n, i);
        if (v != QS_OK) return v;
    }
    return QS_OK;
}

}  // namespace

namespace qs {

// Prepared runs of recently seen circuits: the plan choice and the fused program are pure
// functions of (gates, n, dtype, plan request), so a repeated call reuses them instead of
// planning again.  Keyed by those inputs byte for byte; a small first-in first-out set.
namespace {
struct PrepCache {
    std::mutex mu;
    std::vector<std::pair<std::string, std::shared_ptr<const TrajPrep>>> entries;
    static constexpr size_t kMax = 16;
};
PrepCache &prep_cache()
{
    static PrepCache c;
    return c;
}
std::string prep_key(const qs_gate *gates, int n_gates, int n, qs_dtype dt, const qs_plan *plan)
{
    const qs_plan pl = plan ? *plan : qs_plan{-1, 0, 0, 0, 0};
    const int32_t head[9] = {n, (int32_t)dt, n_gates, pl.fuse, pl.tile_bits, pl.reg_bits, pl.run_bits, pl.mfma,
                             plan ? 1 : 0};
    std::string k((const char *)head, sizeof head);
    if (n_gates > 0) k.append((const char *)gates, sizeof(qs_gate) * (size_t)n_gates);
    return k;
}
}  // namespace

qs_status traj_prepare_shared(const qs_gate *gates, int n_gates, int n, qs_dtype dt, const qs_plan *plan,
                              std::shared_ptr<const TrajPrep> &prep)
{
    if (n < 1 || n > 34) return fail(QS_EINVAL, "run_trajectories: n_qubits must be in 1..34");
    if (dt != QS_C64 && dt != QS_C128) return fail(QS_EINVAL, "run_trajectories: unknown dtype");
    qs_status v = check_circuit(gates, n_gates, n);
    if (v != QS_OK) return v;
    const std::string key = prep_key(gates, n_gates, n, dt, plan);
    {
        PrepCache &c = prep_cache();
        std::lock_guard<std::mutex> lk(c.mu);
        for (auto &e : c.entries)
            if (e.first == key) {
                prep = e.second;
                return QS_OK;
            }
    }
    auto fresh = std::make_shared<TrajPrep>();
    v = traj_prepare_uncached(gates, n_gates, n, dt, plan, *fresh);
    if (v != QS_OK) return v;
    prep = fresh;
    PrepCache &c = prep_cache();
    std::lock_guard<std::mutex> lk(c.mu);
    if (c.entries.size() >= PrepCache::kMax) c.entries.erase(c.entries.begin());
    c.entries.emplace_back(key, prep);
    return QS_OK;
}

qs_status traj_prepare(const qs_gate *gates, int n_gates, int n, qs_dtype dt, const qs_plan *plan,
                       TrajPrep &prep)
{
    std::shared_ptr<const TrajPrep> sp;
    qs_status v = traj_prepare_shared(gates, n_gates, n, dt, plan, sp);
    if (v == QS_OK) prep = *sp;
    return v;
}

static void build_prog_image(TrajPrep &prep);

qs_status traj_prepare_uncached(const qs_gate *gates, int n_gates, int n, qs_dtype dt, const qs_plan *plan,
                                TrajPrep &prep)
{
    qs_status v;
    Plan pl;
    if ((v = resolve_plan(gates, n_gates, n, dt, 1, plan, pl)) != QS_OK) return v;
    prep.n = n;
    prep.dt = dt;
    prep.fused = pl.fused;
    prep.K = pl.K;
    prep.RB = pl.RB;
    prep.prog = std::move(pl.prog);
    // device copy of the gates; CNOTs carry their permutation matrix for fused U2 ops
    prep.hg.assign(gates, gates + n_gates);
    for (auto &g : prep.hg)
        if (g.kind == QS_G_CNOT) std::memcpy(g.m, kCnot4, sizeof kCnot4);
    prep.layout.resize(n);
    for (int q = 0; q < n; ++q) prep.layout[q] = prep.fused ? prep.prog.layout[q] : q;
    if (prep.fused) build_prog_image(prep);
    return QS_OK;
}

static TrajLayout prep_layout(const TrajPrep &prep, int T)
{
    Plan pl;
    pl.fused = prep.fused;
    // only the table sizes of the program enter the layout
    pl.prog.passes.resize(prep.prog.passes.size());
    pl.prog.stages.resize(prep.prog.stages.size());
    pl.prog.rounds.resize(prep.prog.rounds.size());
    pl.prog.ops.resize(prep.prog.ops.size());
    pl.prog.prefs.resize(prep.prog.prefs.size());
    pl.prog.jobs.resize(prep.prog.jobs.size());
    pl.prog.obits.resize(prep.prog.obits.size());
    pl.prog.chain_gates.resize(prep.prog.chain_gates.size());
    pl.prog.chain_off.resize(prep.prog.chain_off.size());
    pl.prog.max_rec = prep.prog.max_rec;
    pl.prog.max_jobs = prep.prog.max_jobs;
    pl.prog.K = prep.prog.K;
    return traj_layout(prep.n, prep.dt, T, (int)prep.hg.size(), pl);
}

size_t traj_prep_bytes(const TrajPrep &prep, int T)
{
    return T < 1 ? 0 : prep_layout(prep, T).total;
}

// The fused program's tables (passes, stages, rounds, ops, input-phase references, outer jobs,
// outer bits, phase chains) laid out as in the run buffer from L.passes on, padding zeroed.
static size_t prog_image_end(const TrajPrep &prep, const TrajLayout &L)
{
    const Program &P = prep.prog;
    return L.chains + sizeof(int32_t) * (P.chain_off.size() + P.chain_gates.size());
}

static void build_prog_image(TrajPrep &prep)
{
    const TrajLayout L = prep_layout(prep, 1);
    const Program &P = prep.prog;
    prep.prog_image.assign(prog_image_end(prep, L) - L.passes, 0);
    char *I = prep.prog_image.data() - L.passes;
    auto put = [&](size_t at, const void *src, size_t bytes) {
        if (bytes) std::memcpy(I + at, src, bytes);
    };
    put(L.passes, P.passes.data(), sizeof(PassDesc) * P.passes.size());
    put(L.stages, P.stages.data(), sizeof(StageDesc) * P.stages.size());
    put(L.rounds, P.rounds.data(), sizeof(RoundDesc) * P.rounds.size());
    put(L.ops, P.ops.data(), sizeof(OpDesc) * P.ops.size());
    put(L.prefs, P.prefs.data(), sizeof(PrepRef) * P.prefs.size());
    put(L.jobs, P.jobs.data(), sizeof(OuterJob) * P.jobs.size());
    put(L.obits, P.obits.data(), sizeof(int32_t) * P.obits.size());
    put(L.chains, P.chain_off.data(), sizeof(int32_t) * P.chain_off.size());
    put(L.chains + sizeof(int32_t) * P.chain_off.size(), P.chain_gates.data(), sizeof(int32_t) * P.chain_gates.size());
}

// Host-to-device copies of the gates and the fused program (the host arrays stay in prep): two
// copies, the gates and the program image, whatever the number of tables.
static qs_status upload_program(const TrajPrep &prep, const TrajLayout &L, char *B, hipStream_t st)
{
    const int n_gates = (int)prep.hg.size();
    if (n_gates > 0)
        QS_HIP(hipMemcpyAsync(B + L.gates, prep.hg.data(), sizeof(qs_gate) * n_gates, hipMemcpyHostToDevice, st));
    if (!prep.fused) return QS_OK;
    QS_HIP(hipMemcpyAsync(B + L.passes, prep.prog_image.data(), prep.prog_image.size(), hipMemcpyHostToDevice, st));
    return QS_OK;
}

// Noise table, initial state, the circuit (fused passes or per-gate sweeps) and the FP64
// reductions into L.out.  With dyn non-null the seed, request, trajectory base, initial index
// and marked index come from device memory (captured graphs).
static qs_status enqueue_compute(const TrajPrep &prep, const TrajLayout &L, char *B, int S, uint64_t init_index,
                                 int64_t pmarked, const qs_noise *nz, const RunParams *dyn, hipStream_t st)
{
    const int n = prep.n;
    const qs_dtype dt = prep.dt;
    const int n_gates = (int)prep.hg.size();
    void *psi = B + L.states;
    double *tab = (double *)(B + L.tab);
    qs_gate *gdev = (qs_gate *)(B + L.gates);
    const Program &P = prep.prog;
    NoiseArgs na{};
    na.dyn = dyn;
    na.e = 0.0;
    na.e_dev = (double *)(B + L.edev);
    na.seed = nz ? nz->seed : 0;
    na.request = nz ? nz->request : 0;
    na.traj_base = nz ? nz->traj_base : 0;
    na.first_noisy_slot = 1;
    QS_HIP(launch_noise_table(gdev, n_gates, S, na, tab, st));
    if (prep.fused && !P.chain_off.empty()) {
        const int32_t *off = (const int32_t *)(B + L.chains);
        QS_HIP(launch_phase_chains(tab, S, off + P.chain_off.size(), off, (int)P.chain_off.size() - 1, st));
    }
    // fused runs make the initial state inside their first pass
    if (!prep.fused || P.passes.empty()) QS_HIP(launch_init_basis(psi, dt, n, S, init_index, st, dyn));
    if (prep.fused) {
        ProgramDev pdv{(const PassDesc *)(B + L.passes), (const StageDesc *)(B + L.stages),
                       (const RoundDesc *)(B + L.rounds), (const OpDesc *)(B + L.ops),
                       (const PrepRef *)(B + L.prefs), (const OuterJob *)(B + L.jobs),
                       (const int32_t *)(B + L.obits)};
        for (size_t p = 0; p < P.passes.size(); ++p) {
            const int64_t init = p == 0 ? (int64_t)init_index : -1;
            uint64_t *otab = (uint64_t *)(B + L.wtab);
            char *wtab = B + L.wtab + align256((size_t(1) << (n > P.K ? n - P.K : 0)) * sizeof(uint64_t));
            QS_HIP(launch_pass_prep(dt, S, &P.passes[p], pdv, tab, gdev, B + L.rec, (int64_t)init_index, dyn, st));
            bool blocks = false;
            for (int ri = P.passes[p].round_begin; ri < P.passes[p].round_end; ++ri)
                blocks = blocks || P.rounds[ri].block_rec >= 0;
            if (blocks) QS_HIP(launch_block_prep(dt, S, &P.passes[p], pdv, B + L.rec, st));
            QS_HIP(launch_pass_jobs(dt, n, S, &P.passes[p], pdv, B + L.rec, init, (int64_t)init_index, dyn,
                                    wtab, otab, st));
            if (p + 1 < P.passes.size()) {
                QS_HIP(launch_fused_pass(psi, dt, n, S, &P.passes[p], (int)p, init, (int64_t)init_index, pdv,
                                         B + L.rec, wtab, otab, st, dyn));
                continue;
            }
            double *part = (double *)(B + L.partials);
            // Small states whose last pass covers few tiles per slot: slot 0 alone would keep a
            // handful of workgroups busy for the whole pass while the rest of the chip idles, so
            // every slot runs in one launch and the overlaps are summed from the stored states
            // (at most 64 KiB per slot).  The choice depends on n and the plan only, never on the
            // number of slots, so a trajectory's results do not depend on its batch.
            const size_t slot_bytes = ((size_t)1 << n) * (dt == QS_C64 ? 8 : 16);
            if (S > 1 && fused_walked_bits(n, &P.passes[p], init) < 8 && slot_bytes <= (64u << 10)) {
                QS_HIP(launch_fused_pass(psi, dt, n, S, &P.passes[p], (int)p, init, (int64_t)init_index, pdv,
                                         B + L.rec, wtab, otab, st, dyn));
                QS_HIP(launch_overlaps(psi, 0, psi, dt, n, S, pmarked, part, (double *)(B + L.out), st, dyn));
                return QS_OK;
            }
            // otherwise the last pass also forms the overlaps with slot 0: slot 0 first, then the
            // others
            QS_HIP(launch_fused_pass(psi, dt, n, S, &P.passes[p], (int)p, init, (int64_t)init_index, pdv, B + L.rec,
                                     wtab, otab, st, dyn, part, 0, 1));
            if (S > 1)
                QS_HIP(launch_fused_pass(psi, dt, n, S, &P.passes[p], (int)p, init, (int64_t)init_index, pdv,
                                         B + L.rec, wtab, otab, st, dyn, part, 1, S - 1));
            QS_HIP(launch_overlap_final(psi, dt, n, S, fused_walked_bits(n, &P.passes[p], init), pmarked, part,
                                        (double *)(B + L.out), st, dyn));
            return QS_OK;
        }
    } else {
        for (int g = 0; g < n_gates; ++g) {
            const qs_gate &G = prep.hg[g];
            const double *row = tab + (size_t)g * S * 8;
            switch (G.kind) {
            case QS_G_U1: QS_HIP(launch_sweep_u1(psi, dt, n, S, G.q0, row, st)); break;
            case QS_G_CP: QS_HIP(launch_sweep_cp(psi, dt, n, S, G.q0, G.q1, row, st)); break;
            case QS_G_SWAP:
            case QS_G_CNOT: QS_HIP(launch_sweep_perm(psi, dt, n, S, G.kind, G.q0, G.q1, st)); break;
            case QS_G_U2: QS_HIP(launch_sweep_2q(psi, dt, n, S, G.q0, G.q1, G.m, st)); break;
            case QS_G_FLIP: QS_HIP(launch_flip(psi, dt, n, S, G.mask, G.value, st)); break;
            case QS_G_DIAG: QS_HIP(launch_scale_pattern(psi, dt, n, S, G.mask, G.value, G.m[0], G.m[1], st)); break;
            }
        }
    }
    QS_HIP(launch_overlaps(psi, 0, psi, dt, n, S, pmarked, (double *)(B + L.partials), (double *)(B + L.out), st,
                           dyn));
    return QS_OK;
}

static int64_t physical_marked(const TrajPrep &prep, int64_t marked)
{
    if (marked < 0) return -1;
    int64_t pm = 0;
    for (int q = 0; q < prep.n; ++q)
        if ((marked >> q) & 1) pm |= (int64_t)1 << prep.layout[q];
    return pm;
}

qs_status traj_launch(const TrajPrep &prep, uint64_t init_index, const qs_noise *nz, int T, int64_t marked,
                      void *dev_buf, size_t buf_bytes, hipStream_t st, double *host_out, TrajRun &run)
{
    const int n = prep.n;
    if (T < 1) return fail(QS_EINVAL, "run_trajectories: n_traj must be >= 1");
    if (init_index >= (1ull << n)) return fail(QS_EINVAL, "run_trajectories: init_index out of range");
    if (marked >= (int64_t)(1ull << n)) return fail(QS_EINVAL, "run_trajectories: marked out of range");
    if (!dev_buf || !aligned256(dev_buf))
        return fail(QS_EINVAL, "run_trajectories: buffer must be non-NULL and 256-byte aligned");
    qs_status v = check_noise(nz, T);
    if (v != QS_OK) return v;
    TrajLayout L = prep_layout(prep, T);
    if (buf_bytes < L.total)
        return fail(QS_EINVAL, "run_trajectories: buffer too small (need " + std::to_string(L.total) + " bytes)");

    char *B = (char *)dev_buf;
    const int S = T + 1;
    run.T = T;
    run.he.assign(S, 0.0);
    for (int t = 0; t < T; ++t) run.he[t + 1] = nz ? (nz->e_per_traj ? nz->e_per_traj[t] : nz->e) : 0.0;
    if ((v = upload_program(prep, L, B, st)) != QS_OK) return v;
    QS_HIP(hipMemcpyAsync(B + L.edev, run.he.data(), sizeof(double) * S, hipMemcpyHostToDevice, st));
    if ((v = enqueue_compute(prep, L, B, S, init_index, physical_marked(prep, marked), nz, nullptr, st)) != QS_OK)
        return v;
    if (host_out) {
        run.host = host_out;
    } else {
        run.host_own.resize((size_t)S * 5);
        run.host = run.host_own.data();
    }
    QS_HIP(hipMemcpyAsync(run.host, B + L.out, sizeof(double) * S * 5, hipMemcpyDeviceToHost, st));
    return QS_OK;
}

void traj_finalize(const TrajPrep &prep, const TrajRun &run, double *fid_out, double *p_out, double *norm_out,
                   int32_t *layout_out)
{
    const double *h = run.host;
    const double n0 = h[2];
    for (int t = 0; t < run.T; ++t) {
        const double *o = &h[(size_t)(t + 1) * 5];
        if (fid_out) fid_out[t] = (o[0] * o[0] + o[1] * o[1]) / (n0 * o[2]);
        if (p_out) p_out[t] = o[3] * o[3] + o[4] * o[4];
        if (norm_out) norm_out[t] = o[2];
    }
    if (layout_out)
        for (int q = 0; q < prep.n; ++q) layout_out[q] = prep.layout[q];
}

}  // namespace qs

extern "C" {

size_t qs_traj_bytes_required(const qs_gate *gates, int n_gates, int n, qs_dtype dt, int T,
                              const qs_plan *plan)
{
    if (n < 1 || n > 34 || T < 1 || (dt != QS_C64 && dt != QS_C128)) return 0;
    // the run's own (cached) preparation: a repeated call neither plans nor prices the shapes again
    std::shared_ptr<const TrajPrep> prep;
    if (traj_prepare_shared(gates, n_gates, n, dt, plan, prep) != QS_OK) return 0;
    return traj_prep_bytes(*prep, T);
}

qs_status qs_traj_layout(const qs_gate *gates, int n_gates, int n, qs_dtype dt, int T, const qs_plan *plan,
                         size_t *out)
{
    clear_error();
    if (!out) return fail(QS_EINVAL, "traj_layout: out is NULL");
    if (n < 1 || n > 34 || T < 1 || (dt != QS_C64 && dt != QS_C128))
        return fail(QS_EINVAL, "traj_layout: bad size or dtype");
    std::shared_ptr<const TrajPrep> prep;
    qs_status v = traj_prepare_shared(gates, n_gates, n, dt, plan, prep);
    if (v != QS_OK) return v;
    TrajLayout L = prep_layout(*prep, T);
    size_t vals[17] = {L.states, L.tab, L.gates, L.edev, L.passes, L.stages, L.rounds, L.ops, L.prefs,
                       L.jobs, L.obits, L.chains, L.wtab, L.rec, L.partials, L.out, L.total};
    for (int i = 0; i < 17; ++i) out[i] = vals[i];
    return QS_OK;
}

qs_status qs_plan_choose(const qs_gate *gates, int n_gates, int n, qs_dtype dt, qs_plan *out,
                         double *model_s_per_slot)
{
    clear_error();
    if (!out) return fail(QS_EINVAL, "plan_choose: out is NULL");
    if (n < 1 || n > 34) return fail(QS_EINVAL, "plan_choose: n_qubits must be in 1..34");
    if (dt != QS_C64 && dt != QS_C128) return fail(QS_EINVAL, "plan_choose: unknown dtype");
    qs_status v = check_circuit(gates, n_gates, n);
    if (v != QS_OK) return v;
    Plan pl;
    double cost = 0.0;
    if ((v = autotune_plan(gates, n_gates, n, dt, kModelSlots, pl, &cost)) != QS_OK) return v;
    out->fuse = pl.fused ? 1 : 0;
    out->tile_bits = pl.fused ? pl.K : 0;
    out->reg_bits = pl.fused ? pl.RB : 0;
    out->run_bits = pl.fused ? pl.run_bits : 0;
    out->mfma = pl.fused && pl.mfma ? 1 : 0;
    if (model_s_per_slot) *model_s_per_slot = cost;
    return QS_OK;
}

qs_status qs_plan_describe(const qs_gate *gates, int n_gates, int n, qs_dtype dt, const qs_plan *plan,
                           char *buf, size_t cap, size_t *len)
{
    clear_error();
    if (n < 1 || n > 34) return fail(QS_EINVAL, "plan_describe: n_qubits must be in 1..34");
    if (dt != QS_C64 && dt != QS_C128) return fail(QS_EINVAL, "plan_describe: unknown dtype");
    qs_status v = check_circuit(gates, n_gates, n);
    if (v != QS_OK) return v;
    Plan pl;
    if ((v = resolve_plan(gates, n_gates, n, dt, 1, plan, pl)) != QS_OK) return v;
    std::string o;
    auto I = [&](const char *k, long long x) { o += "\""; o += k; o += "\":" + std::to_string(x) + ","; };
    o += "{";
    I("fused", pl.fused ? 1 : 0);
    I("K", pl.prog.K);
    I("RB", pl.prog.RB);
    I("mfma", pl.mfma ? 1 : 0);
    I("run_bits", pl.run_bits);
    if (pl.fused) I("stage_rec_cap", stage_rec_cap(dt, pl.prog.K));
    {
        const double cost = pl.fused ? model_cost_fused(pl.prog, n, dt, kModelSlots, pl.run_bits)
                                     : model_cost_unfused(gates, n_gates, n, dt, kModelSlots);
        char b[64];
        std::snprintf(b, sizeof b, "\"model_s_per_slot\":%.6e,", cost);
        o += b;
    }
    o += "\"layout\":[";
    for (size_t q = 0; q < pl.prog.layout.size(); ++q) o += (q ? "," : "") + std::to_string(pl.prog.layout[q]);
    o += "],\"chains\":[";
    for (size_t c = 0; c + 1 < pl.prog.chain_off.size(); ++c) {
        o += c ? ",[" : "[";
        for (int k = pl.prog.chain_off[c]; k < pl.prog.chain_off[c + 1]; ++k)
            o += (k != pl.prog.chain_off[c] ? "," : "") + std::to_string(pl.prog.chain_gates[k]);
        o += "]";
    }
    o += "],\"passes\":[";
    const Program &P = pl.prog;
    for (size_t pi = 0; pi < P.passes.size(); ++pi) {
        const PassDesc &pd = P.passes[pi];
        o += pi ? ",{" : "{";
        o += "\"q_pos\":[";
        for (int j = 0; j < pd.K; ++j) o += (j ? "," : "") + std::to_string(pd.q_pos[j]);
        o += "],";
        I("outer_mask", (long long)pd.outer_mask);
        I("classical", (long long)pd.classical);
        I("lclassical", (long long)pd.lclassical);
        I("zero_fill", pd.zero_fill);
        I("uni_kernel", pd.uni_kernel);
        I("zin_ops", pd.zin_ops);
        I("mixed_ops", pd.mixed_ops);
        I("rec_size", pd.rec_size);
        I("load_round", pd.load_round);
        I("load_reg_mask", P.rounds[pd.load_round].reg_mask);
        I("store_round", pd.store_round);
        I("blocks", pd.blocks);
        I("store_reg_mask", P.rounds[pd.store_round].reg_mask);
        I("round_begin", pd.round_begin);
        I("round_end", pd.round_end);
        I("op_begin", pd.op_begin);
        I("op_end", pd.op_end);
        I("job_begin", pd.job_begin);
        I("job_end", pd.job_end);
        o += "\"stages\":[";
        for (int si = pd.stage_begin; si < pd.stage_end; ++si) {
            const StageDesc &sd = P.stages[si];
            o += si != pd.stage_begin ? ",{" : "{";
            I("rec_begin", sd.rec_begin);
            I("rec_end", sd.rec_end);
            I("round_begin", sd.round_begin);
            I("op_begin", sd.op_begin);
            I("job_begin", sd.job_begin);
            I("job_end", sd.job_end);
            I("n_jobs", sd.job_end - sd.job_begin);
            o += "\"rounds\":[";
            for (int ri = sd.round_begin; ri < sd.round_end; ++ri) {
                const RoundDesc &rd = P.rounds[ri];
                o += ri != sd.round_begin ? ",{" : "{";
                I("reg_mask", rd.reg_mask);
                I("block_rec", rd.block_rec);
                I("seq", rd.seq);
                o += "\"ops\":[";
                for (int oi = rd.op_begin; oi < rd.op_end; ++oi) {
                    const OpDesc &op = P.ops[oi];
                    o += oi != rd.op_begin ? ",{" : "{";
                    I("type", op.type);
                    I("flags", op.flags);
                    I("creg", op.creg);
                    I("p0", op.p0);
                    I("p1", op.p1);
                    I("gate", op.gate);
                    I("rec", op.rec);
                    I("diag_kind", op.diag_kind);
                    I("lmask", op.lmask);
                    I("lvalue", op.lvalue);
                    I("omask", (long long)op.omask);
                    I("ovalue", (long long)op.ovalue);
                    o += "\"phases\":[";
                    for (int k = op.pref_begin; k < op.pref_end; ++k) {
                        const PrepRef &pr = P.prefs[k];
                        o += (k != op.pref_begin ? ",[" : "[") + std::to_string(pr.kind) + "," +
                             std::to_string(pr.post) + "," + std::to_string(pr.bit) + "," +
                             std::to_string(pr.gate) + "]";
                    }
                    o += "]}";
                }
                o += "]}";
            }
            o += "]}";
        }
        o += "]}";
    }
    o += "]}";
    if (len) *len = o.size();
    if (buf && cap > 0) {
        size_t k = std::min(cap - 1, o.size());
        std::memcpy(buf, o.data(), k);
        buf[k] = 0;
    }
    return QS_OK;
}

qs_status qs_run_trajectories(const qs_gate *gates, int n_gates, int n, uint64_t init_index, qs_dtype dt,
                              const qs_noise *nz, int T, int64_t marked, const qs_plan *plan,
                              void *dev_buf, size_t buf_bytes, void *hip_stream, double *fid_out,
                              double *p_out, double *norm_out, int32_t *layout_out)
{
    clear_error();
    if (!fid_out) return fail(QS_EINVAL, "run_trajectories: fid_out is NULL");
    if (p_out && marked < 0) return fail(QS_EINVAL, "run_trajectories: p_out needs marked >= 0");
    if (T < 1) return fail(QS_EINVAL, "run_trajectories: n_traj must be >= 1");
    std::shared_ptr<const qs::TrajPrep> prep;   // keeps the host arrays alive until the copies are done
    qs_status v = qs::traj_prepare_shared(gates, n_gates, n, dt, plan, prep);
    if (v != QS_OK) return v;
    qs::TrajRun run;
    if ((v = qs::traj_launch(*prep, init_index, nz, T, marked, dev_buf, buf_bytes, (hipStream_t)hip_stream,
                             nullptr, run)) != QS_OK)
        return v;
    QS_HIP(hipStreamSynchronize((hipStream_t)hip_stream));
    qs::traj_finalize(*prep, run, fid_out, p_out, norm_out, layout_out);
    return QS_OK;
}

// ---------------------------------------------------------------------------------------
// Density-matrix runs (Section 3) through the trajectory machinery
// ---------------------------------------------------------------------------------------
namespace qs {
namespace {

// The gates of a noisy n-qubit circuit as a noiseless circuit on vec(rho) (2n qubits, entry
// rho_ij at index i 2^n + j): the circuit's channels one after another, each as a gate list
// on the row bits (q + n) and the column bits (q).
//   * one-qubit U with ROT noise and e > 0: its eq. (6) Kraus pair {U E1, U E2} as one dense
//     two-qubit gate on (column bit q, row bit q + n), M[b + 2a][b' + 2a'] =
//     sum_k K_k[a][a'] conj(K_k[b][b']);
//   * controlled phase with PHASE noise and e > 0: the averaged channel of eq. (9), entry rho_ij
//     times exp(-i theta (b_i - b_j)) exp(-e^2 (b_i - b_j)^2 / 2) (b = both qubits 1), as three
//     diagonal patterns: rows with b_i = 1 by exp(-i theta) exp(-e^2/2), columns with b_j = 1
//     by exp(i theta) exp(-e^2/2), entries with both by exp(e^2);
//   * every other gate G (and the noisy ones at e = 0): G on the row bits, conj(G) on the
//     column bits (SWAP, CNOT and FLIP are real).
void dm_superop_gates(const qs_gate *gates, int n_gates, int n, double e, std::vector<qs_gate> &out)
{
    out.clear();
    out.reserve((size_t)n_gates * 2);
    for (int gi = 0; gi < n_gates; ++gi) {
        const qs_gate &G = gates[gi];
        qs_gate ket = G, bra = G;
        ket.noise = bra.noise = QS_NOISE_NONE;
        if (G.kind == QS_G_U1 && e > 0 && G.noise == QS_NOISE_ROT) {
            double ops[16];
            kraus_rot_ops(G.m, e, ops);
            qs_gate s{};
            s.kind = QS_G_U2;
            s.q0 = G.q0;
            s.q1 = G.q0 + n;
            s.site = G.site;
            for (int l = 0; l < 4; ++l)
                for (int lp = 0; lp < 4; ++lp) {
                    const int b = l & 1, a = l >> 1, bp = lp & 1, ap = lp >> 1;
                    std::complex<double> v = 0;
                    for (int k = 0; k < 2; ++k) {
                        const double *K = ops + 8 * k;
                        std::complex<double> ka(K[4 * a + 2 * ap], K[4 * a + 2 * ap + 1]);
                        std::complex<double> kb(K[4 * b + 2 * bp], K[4 * b + 2 * bp + 1]);
                        v += ka * std::conj(kb);
                    }
                    s.m[2 * (4 * l + lp)] = v.real();
                    s.m[2 * (4 * l + lp) + 1] = v.imag();
                }
            out.push_back(s);
            continue;
        }
        if (G.kind == QS_G_CP && e > 0 && G.noise == QS_NOISE_PHASE) {
            const uint64_t cm = (1ull << G.q0) | (1ull << G.q1);
            const double sp = std::exp(-0.5 * e * e);
            qs_gate d{};
            d.kind = QS_G_DIAG;
            d.site = G.site;
            d.mask = d.value = cm << n;
            d.m[0] = std::cos(G.theta) * sp;
            d.m[1] = -std::sin(G.theta) * sp;
            out.push_back(d);
            d.mask = d.value = cm;
            d.m[1] = -d.m[1];
            out.push_back(d);
            d.mask = d.value = cm | (cm << n);
            d.m[0] = std::exp(e * e);
            d.m[1] = 0.0;
            out.push_back(d);
            continue;
        }
        switch (G.kind) {
        case QS_G_U1:
            ket.q0 += n;
            for (int k = 1; k < 8; k += 2) bra.m[k] = -G.m[k];
            break;
        case QS_G_CP:
            ket.q0 += n;
            ket.q1 += n;
            bra.theta = -G.theta;
            break;
        case QS_G_SWAP:
        case QS_G_CNOT:
            ket.q0 += n;
            ket.q1 += n;
            break;
        case QS_G_U2:
            ket.q0 += n;
            ket.q1 += n;
            for (int k = 1; k < 32; k += 2) bra.m[k] = -G.m[k];
            break;
        case QS_G_FLIP:
            ket.mask <<= n;
            ket.value <<= n;
            break;
        case QS_G_DIAG:
            ket.mask <<= n;
            ket.value <<= n;
            bra.m[1] = -G.m[1];
            break;
        }
        out.push_back(ket);
        out.push_back(bra);
    }
}

// Buffer of a density-matrix run: the trajectory layout of the superoperator circuit with
// one slot (vec(rho)), then psi in the run's physical bit order, the expectation partials and
// its four output doubles.
struct DmLayout {
    TrajLayout L;
    size_t psi, partials, out, total;
};

DmLayout dm_layout(const TrajPrep &prep, int n)
{
    DmLayout D{};
    D.L = prep_layout(prep, 0);
    size_t off = D.L.total;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off = align256(off + bytes);
        return at;
    };
    D.psi = take(state_bytes(n, prep.dt, 1));
    D.partials = take(reduce_partials_doubles(n, 1) * sizeof(double));
    D.out = take(16 * sizeof(double));
    D.total = off;
    return D;
}

qs_status dm_prepare(const qs_gate *gates, int n_gates, int n, qs_dtype dt, double e, const qs_plan *plan,
                     TrajPrep &prep)
{
    if (n < 1 || 2 * n > 34) return fail(QS_EINVAL, "dm_run: n_qubits must be in 1..17");
    if (!std::isfinite(e) || e < 0) return fail(QS_EINVAL, "dm_run: e must be finite and >= 0");
    qs_status v = check_circuit(gates, n_gates, n);
    if (v != QS_OK) return v;
    std::vector<qs_gate> sg;
    dm_superop_gates(gates, n_gates, n, e, sg);
    return traj_prepare(sg.data(), (int)sg.size(), 2 * n, dt, plan, prep);
}

}  // namespace
}  // namespace qs

extern "C" {

qs_status qs_dm_superop(const qs_gate *gates, int n_gates, int n_qubits, double e, qs_gate *out, int cap,
                        int *n_out)
{
    clear_error();
    if (!n_out) return fail(QS_EINVAL, "dm_superop: n_out is NULL");
    *n_out = 0;
    if (n_qubits < 1 || 2 * n_qubits > 34) return fail(QS_EINVAL, "dm_superop: n_qubits must be in 1..17");
    if (!std::isfinite(e) || e < 0) return fail(QS_EINVAL, "dm_superop: e must be finite and >= 0");
    qs_status v = check_circuit(gates, n_gates, n_qubits);
    if (v != QS_OK) return v;
    std::vector<qs_gate> sg;
    qs::dm_superop_gates(gates, n_gates, n_qubits, e, sg);
    *n_out = (int)sg.size();
    if (!out) return QS_OK;
    if (cap < (int)sg.size())
        return fail(QS_EINVAL, "dm_superop: cap below the " + std::to_string(sg.size()) + " gates of the result");
    std::copy(sg.begin(), sg.end(), out);
    return QS_OK;
}

size_t qs_dm_run_bytes_required(const qs_gate *gates, int n_gates, int n_qubits, qs_dtype dt, double e,
                                const qs_plan *plan)
{
    clear_error();
    qs::TrajPrep prep;
    if (qs::dm_prepare(gates, n_gates, n_qubits, dt, e, plan, prep) != QS_OK) return 0;
    return qs::dm_layout(prep, n_qubits).total;
}

qs_status qs_dm_run(const qs_gate *gates, int n_gates, int n_qubits, uint64_t init_index, qs_dtype dt, double e,
                    const qs_plan *plan, const void *psi_dev, void *dev_buf, size_t buf_bytes, void *hip_stream,
                    double *f_out, double *trace_out, int32_t *layout_out)
{
    clear_error();
    if (!psi_dev || !f_out) return fail(QS_EINVAL, "dm_run: psi_dev and f_out must be non-NULL");
    if (!dev_buf || !qs::aligned256(dev_buf))
        return fail(QS_EINVAL, "dm_run: buffer must be non-NULL and 256-byte aligned");
    const int n = n_qubits;
    qs::TrajPrep prep;
    qs_status v = qs::dm_prepare(gates, n_gates, n, dt, e, plan, prep);
    if (v != QS_OK) return v;
    if (init_index >= (1ull << n)) return fail(QS_EINVAL, "dm_run: init_index out of range");
    const qs::DmLayout D = qs::dm_layout(prep, n);
    if (buf_bytes < D.total)
        return fail(QS_EINVAL, "dm_run: buffer too small (need " + std::to_string(D.total) + " bytes)");
    // SWAPs act on the row and the column bits alike, so the relabelling keeps the two halves
    // apart and permutes them the same way
    std::vector<int32_t> sigma(n);
    bool identity = true;
    for (int q = 0; q < n; ++q) {
        sigma[q] = prep.layout[q];
        if (prep.layout[q + n] != prep.layout[q] + n || prep.layout[q] < 0 || prep.layout[q] >= n)
            return fail(QS_EUNSUPPORTED, "dm_run: the plan's relabelling mixes row and column bits");
        identity = identity && sigma[q] == q;
    }
    hipStream_t st = (hipStream_t)hip_stream;
    char *B = (char *)dev_buf;
    if ((v = qs::upload_program(prep, D.L, B, st)) != QS_OK) return v;
    const double zero = 0.0;
    QS_HIP(hipMemcpyAsync(B + D.L.edev, &zero, sizeof zero, hipMemcpyHostToDevice, st));
    const uint64_t init = (init_index << n) | init_index;
    if ((v = qs::enqueue_compute(prep, D.L, B, 1, init, -1, nullptr, nullptr, st)) != QS_OK) return v;
    const void *psi_phys = psi_dev;
    if (!identity) {
        QS_HIP(qs::launch_permute_bits(B + D.psi, psi_dev, dt, n, sigma.data(), st));
        psi_phys = B + D.psi;
    }
    QS_HIP(qs::launch_dm_expect(B + D.L.states, psi_phys, dt, n, (double *)(B + D.partials),
                                (double *)(B + D.out), st));
    double h[4];
    QS_HIP(hipMemcpyAsync(h, B + D.out, sizeof h, hipMemcpyDeviceToHost, st));
    QS_HIP(hipStreamSynchronize(st));
    *f_out = h[0];
    if (trace_out) *trace_out = h[2];
    if (layout_out)
        for (int q = 0; q < n; ++q) layout_out[q] = sigma[q];
    return QS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------
// Captured trajectory runs
// ---------------------------------------------------------------------------------------
struct qs_traj_graph_s {
    qs::TrajPrep prep;
    int T = 0;
    char *buf = nullptr;
    TrajLayout L{};
    int device = 0;
    hipStream_t st = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    double *h_out = nullptr;          // pinned: S * 5 result doubles
    double *h_e = nullptr;            // pinned: S per-slot noise strengths
    RunParams *h_params = nullptr;    // pinned: per-run values
};

static void graph_free(qs_traj_graph_s *g)
{
    if (!g) return;
    if (g->st) (void)hipStreamSynchronize(g->st);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->h_out) (void)hipHostFree(g->h_out);
    if (g->h_e) (void)hipHostFree(g->h_e);
    if (g->h_params) (void)hipHostFree(g->h_params);
    if (g->st) (void)hipStreamDestroy(g->st);
    delete g;
}

qs_status qs_traj_graph_bytes_required(const qs_gate *gates, int n_gates, int n, qs_dtype dt, int T,
                                       const qs_plan *plan, size_t *bytes)
{
    clear_error();
    if (!bytes) return fail(QS_EINVAL, "traj_graph_bytes_required: bytes is NULL");
    if (T < 1) return fail(QS_EINVAL, "traj_graph_bytes_required: n_traj must be >= 1");
    std::shared_ptr<const qs::TrajPrep> prep;
    qs_status v = qs::traj_prepare_shared(gates, n_gates, n, dt, plan, prep);
    if (v != QS_OK) return v;
    *bytes = qs::traj_prep_bytes(*prep, T);
    return QS_OK;
}

qs_status qs_traj_graph_create(const qs_gate *gates, int n_gates, int n, qs_dtype dt, int T, const qs_plan *plan,
                               void *dev_buf, size_t buf_bytes, qs_traj_graph *out)
{
    clear_error();
    if (!out) return fail(QS_EINVAL, "traj_graph_create: out is NULL");
    *out = nullptr;
    if (T < 1) return fail(QS_EINVAL, "traj_graph_create: n_traj must be >= 1");
    if (!dev_buf || !aligned256(dev_buf))
        return fail(QS_EINVAL, "traj_graph_create: buffer must be non-NULL and 256-byte aligned");
    auto *g = new qs_traj_graph_s();
    qs_status v = qs::traj_prepare(gates, n_gates, n, dt, plan, g->prep);
    if (v != QS_OK) {
        delete g;
        return v;
    }
    g->T = T;
    g->L = qs::prep_layout(g->prep, T);
    if (buf_bytes < g->L.total) {
        const size_t need = g->L.total;
        delete g;
        return fail(QS_EINVAL, "traj_graph_create: buffer too small (need " + std::to_string(need) + " bytes)");
    }
    g->buf = (char *)dev_buf;
    const int S = T + 1;
    auto bail = [&](hipError_t e, const char *what) {
        (void)hipGetLastError();
        if (g->st) {
            hipGraph_t partial = nullptr;
            hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
            if (hipStreamIsCapturing(g->st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) {
                (void)hipStreamEndCapture(g->st, &partial);
                if (partial) (void)hipGraphDestroy(partial);
            }
        }
        graph_free(g);
        return hip_fail(e, what);
    };
    hipError_t e;
    if ((e = hipStreamCreateWithFlags(&g->st, hipStreamNonBlocking)) != hipSuccess) return bail(e, "stream");
    if ((e = hipHostMalloc((void **)&g->h_out, sizeof(double) * 5 * S, hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc((void **)&g->h_e, sizeof(double) * S, hipHostMallocDefault)) != hipSuccess ||
        (e = hipHostMalloc((void **)&g->h_params, sizeof(RunParams), hipHostMallocDefault)) != hipSuccess)
        return bail(e, "hipHostMalloc");
    std::memset(g->h_e, 0, sizeof(double) * S);
    std::memset(g->h_params, 0, sizeof(RunParams));
    if ((v = qs::upload_program(g->prep, g->L, g->buf, g->st)) != QS_OK) {
        graph_free(g);
        return v;
    }
    if ((e = hipStreamSynchronize(g->st)) != hipSuccess) return bail(e, "upload");
    if ((e = fused_prepare_attributes()) != hipSuccess) return bail(e, "fused kernel attributes");
    const RunParams *dyn = (const RunParams *)(g->buf + g->L.dyn);
    if ((e = hipStreamBeginCapture(g->st, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return bail(e, "hipStreamBeginCapture");
    if ((e = hipMemcpyAsync(g->buf + g->L.dyn, g->h_params, sizeof(RunParams), hipMemcpyHostToDevice, g->st)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(g->buf + g->L.edev, g->h_e, sizeof(double) * S, hipMemcpyHostToDevice, g->st)) !=
            hipSuccess)
        return bail(e, "capture copies");
    // kernel arguments that dyn overrides carry placeholders: the first pass is always a
    // making pass (init 0) and the marked amplitude is read when dyn->marked >= 0
    if ((v = qs::enqueue_compute(g->prep, g->L, g->buf, S, 0, 0, nullptr, dyn, g->st)) != QS_OK) {
        std::string msg = qs_last_error();
        (void)bail(hipSuccess, "capture");
        return fail(v, msg);
    }
    if ((e = hipMemcpyAsync(g->h_out, g->buf + g->L.out, sizeof(double) * 5 * S, hipMemcpyDeviceToHost, g->st)) !=
        hipSuccess)
        return bail(e, "capture copies");
    if ((e = hipStreamEndCapture(g->st, &g->graph)) != hipSuccess) return bail(e, "hipStreamEndCapture");
    if ((e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0)) != hipSuccess)
        return bail(e, "hipGraphInstantiate");
    *out = g;
    return QS_OK;
}

qs_status qs_traj_graph_launch(qs_traj_graph g, uint64_t init_index, const qs_noise *nz, int64_t marked,
                               double *fid_out, double *p_out, double *norm_out, int32_t *layout_out)
{
    clear_error();
    if (!g || !fid_out) return fail(QS_EINVAL, "traj_graph_launch: NULL graph or fid_out");
    const int n = g->prep.n, T = g->T, S = T + 1;
    if (init_index >= (1ull << n)) return fail(QS_EINVAL, "traj_graph_launch: init_index out of range");
    if (marked >= (int64_t)(1ull << n)) return fail(QS_EINVAL, "traj_graph_launch: marked out of range");
    if (p_out && marked < 0) return fail(QS_EINVAL, "traj_graph_launch: p_out needs marked >= 0");
    qs_status v = check_noise(nz, T);
    if (v != QS_OK) return v;
    // the previous replay has finished (launch blocks), so the pinned inputs are free
    g->h_params->seed = nz ? nz->seed : 0;
    g->h_params->request = nz ? nz->request : 0;
    g->h_params->traj_base = nz ? nz->traj_base : 0;
    g->h_params->init = (int64_t)init_index;
    g->h_params->marked = qs::physical_marked(g->prep, marked);
    g->h_e[0] = 0.0;
    for (int t = 0; t < T; ++t) g->h_e[t + 1] = nz ? (nz->e_per_traj ? nz->e_per_traj[t] : nz->e) : 0.0;
    QS_HIP(hipGraphLaunch(g->exec, g->st));
    QS_HIP(hipStreamSynchronize(g->st));
    qs::TrajRun run;
    run.T = T;
    run.host = g->h_out;
    qs::traj_finalize(g->prep, run, fid_out, p_out, norm_out, layout_out);
    (void)S;
    return QS_OK;
}

qs_status qs_traj_graph_destroy(qs_traj_graph g)
{
    clear_error();
    graph_free(g);
    return QS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------------------
// Fixed rank
// ---------------------------------------------------------------------------------------
namespace {

using cd = std::complex<double>;

// Cyclic Jacobi for a Hermitian m x m matrix (row-major A): on return w holds the eigenvalues
// and the columns of Vec the eigenvectors.  Each rotation first turns A_pq real with a phase
// on column q, then zeroes it with a real plane rotation (Golub & Van Loan, sec. 8.5).
void jacobi_hermitian(int m, std::vector<cd> &A, std::vector<double> &w, std::vector<cd> &Vec)
{
    Vec.assign((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) Vec[(size_t)i * m + i] = 1.0;
    auto at = [&](int i, int j) -> cd & { return A[(size_t)i * m + j]; };
    double fro = 0;
    for (auto &x : A) fro += std::norm(x);
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0;
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < m; ++j)
                if (i != j) off += std::norm(at(i, j));
        if (off <= 1e-32 * fro || off == 0.0) break;
        for (int p = 0; p < m - 1; ++p)
            for (int q = p + 1; q < m; ++q) {
                cd apq = at(p, q);
                double r = std::abs(apq);
                if (r == 0.0) continue;
                cd ph = apq / r;                      // e^{i phi}
                double app = at(p, p).real(), aqq = at(q, q).real();
                double theta = 0.5 * std::atan2(2.0 * r, aqq - app);
                double c = std::cos(theta), s = std::sin(theta);
                cd em = std::conj(ph);                // e^{-i phi}
                // J = D R: J_pp = c, J_pq = s, J_qp = -s e^{-i phi}, J_qq = c e^{-i phi}
                for (int k = 0; k < m; ++k) {         // A <- A J
                    cd akp = at(k, p), akq = at(k, q);
                    at(k, p) = akp * c - akq * s * em;
                    at(k, q) = akp * s + akq * c * em;
                }
                for (int k = 0; k < m; ++k) {         // A <- J^dagger A
                    cd apk = at(p, k), aqk = at(q, k);
                    at(p, k) = apk * c - aqk * s * ph;
                    at(q, k) = apk * s + aqk * c * ph;
                }
                at(p, q) = 0.0;
                at(q, p) = 0.0;
                at(p, p) = at(p, p).real();
                at(q, q) = at(q, q).real();
                for (int k = 0; k < m; ++k) {         // Vec <- Vec J
                    cd vkp = Vec[(size_t)k * m + p], vkq = Vec[(size_t)k * m + q];
                    Vec[(size_t)k * m + p] = vkp * c - vkq * s * em;
                    Vec[(size_t)k * m + q] = vkp * s + vkq * c * em;
                }
            }
    }
    w.resize(m);
    for (int i = 0; i < m; ++i) w[i] = at(i, i).real();
}

}  // namespace

extern "C" {

size_t qs_fr_bytes_required(int n, int r, qs_dtype dt)
{
    if (n < 1 || n > 34 || r < 1 || r > 8 || (dt != QS_C64 && dt != QS_C128)) return 0;
    return state_bytes(n, dt, r);
}

qs_status qs_fr_create(int n, int r, qs_dtype dt, void *buf, size_t bytes, void *stream, qs_fr *out)
{
    clear_error();
    if (!out) return fail(QS_EINVAL, "fr_create: out is NULL");
    *out = nullptr;
    if (n < 2 || n > 34) return fail(QS_EINVAL, "fr_create: n_qubits must be in 2..34");
    if (r < 1 || r > 8) return fail(QS_EINVAL, "fr_create: rank bound r must be in 1..8");
    if (dt != QS_C64 && dt != QS_C128) return fail(QS_EINVAL, "fr_create: unknown dtype");
    if (!buf || !aligned256(buf)) return fail(QS_EINVAL, "fr_create: buffer must be non-NULL and 256-byte aligned");
    if (bytes < state_bytes(n, dt, r)) return fail(QS_EINVAL, "fr_create: buffer too small");
    auto *f = new (std::nothrow) qs_fr_s();
    if (!f) return fail(QS_ENOMEM, "fr_create: out of host memory");
    f->n = n;
    f->r = r;
    f->rank = 0;
    f->dt = dt;
    f->V = buf;
    f->st = (hipStream_t)stream;
    f->log_trace = 0.0;
    size_t off = 0;
    off += align256(fr_gram_partials_doubles(n, r) * 8) / 8;
    f->off_gram = off;
    off += kFrHostGram;
    f->off_coef = off;
    off += kFrHostGram;
    f->off_ovp = off;
    off += align256(reduce_partials_doubles(n, 8) * 8) / 8;
    f->off_ovo = off;
    off += 64;
    f->off_tab = off;
    off += 64 + 64;
    hipError_t e = hipMalloc(&f->scratch, off * sizeof(double));
    if (e != hipSuccess) {
        delete f;
        return hip_fail(e, "fr_create: hipMalloc scratch");
    }
    e = hipHostMalloc(&f->host, 2 * kFrHostGram * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipFree(f->scratch);
        delete f;
        return hip_fail(e, "fr_create: hipHostMalloc staging");
    }
    *out = f;
    return QS_OK;
}

qs_status qs_fr_destroy(qs_fr f)
{
    clear_error();
    if (!f) return QS_OK;
    (void)hipStreamSynchronize(f->st);
    (void)hipFree(f->scratch);
    (void)hipHostFree(f->host);
    delete f;
    return QS_OK;
}

qs_status qs_fr_init_basis(qs_fr f, uint64_t index)
{
    clear_error();
    if (!f) return fail(QS_EINVAL, "fr_init_basis: NULL handle");
    if (index >= (1ull << f->n)) return fail(QS_EINVAL, "fr_init_basis: index out of range");
    QS_HIP(launch_init_basis(f->V, f->dt, f->n, 1, index, f->st));
    f->rank = 1;
    f->log_trace = 0.0;
    return QS_OK;
}

qs_status qs_fr_apply_gate(qs_fr f, const qs_gate *g)
{
    clear_error();
    if (!f || !g) return fail(QS_EINVAL, "fr_apply_gate: NULL argument");
    if (f->rank < 1) return fail(QS_EINVAL, "fr_apply_gate: call fr_init_basis first");
    qs_status v = check_gate(*g, f->n, 0);
    if (v != QS_OK) return v;
    return sweep_gate(f->V, f->dt, f->n, f->rank, *g, nullptr, f->scratch + f->off_tab, f->st);
}

}  // extern "C"

// One Kraus step of the fixed-rank form (Section 3.2) for a set on k = 1 or 2 qubits: the Gram
// matrix of the 2^k r sub-columns on the device, G = W^dagger W on the host, its FP64
// eigen-decomposition, the truncation rule, and the recombination of the kept eigenvectors.
static qs_status fr_kraus_step(qs_fr f, int k, const int32_t *qb, int n_ops, const double *ops, double tau,
                               double zero_tol, int *rank_out, const char *who)
{
    const int d = 1 << k;            // operator dimension
    const int G = d * 8;             // sub-columns of the Gram matrix (column c < rank at x * 8 + c)
    const int rin = f->rank;
    double *gram_dev = f->scratch + f->off_gram;
    if (k == 1) QS_HIP(launch_fr_gram(f->V, f->dt, f->n, rin, qb[0], f->scratch, gram_dev, f->st));
    else QS_HIP(launch_fr_gram2(f->V, f->dt, f->n, rin, qb[0], qb[1], f->scratch, gram_dev, f->st));
    QS_HIP(hipMemcpyAsync(f->host, gram_dev, (size_t)G * G * 2 * sizeof(double), hipMemcpyDeviceToHost, f->st));
    QS_HIP(hipStreamSynchronize(f->st));
    // Gamma[(x, c), (y, d)] at index (x * 8 + c) * G + (y * 8 + d)
    auto Gam = [&](int x, int c, int y, int dd) {
        size_t i = (size_t)(x * 8 + c) * G + (y * 8 + dd);
        return cd(f->host[2 * i], f->host[2 * i + 1]);
    };
    const int dd2 = d * d;
    auto E = [&](int a, int r, int c) {
        const size_t i = (size_t)dd2 * a + (size_t)d * r + c;
        return cd(ops[2 * i], ops[2 * i + 1]);
    };
    const int m = n_ops * rin;
    std::vector<cd> GW((size_t)m * m);
    std::vector<cd> C((size_t)dd2);   // (E_a^dagger E_b)[x][y]
    for (int a = 0; a < n_ops; ++a)
        for (int b = 0; b < n_ops; ++b) {
            for (int x = 0; x < d; ++x)
                for (int y = 0; y < d; ++y) {
                    cd acc = 0;
                    for (int z = 0; z < d; ++z) acc += std::conj(E(a, z, x)) * E(b, z, y);
                    C[(size_t)x * d + y] = acc;
                }
            for (int c = 0; c < rin; ++c)
                for (int e2 = 0; e2 < rin; ++e2) {
                    cd acc = 0;
                    for (int x = 0; x < d; ++x)
                        for (int y = 0; y < d; ++y) acc += C[(size_t)x * d + y] * Gam(x, c, y, e2);
                    GW[(size_t)(a * rin + c) * m + (b * rin + e2)] = acc;
                }
        }
    std::vector<double> w;
    std::vector<cd> Q;
    jacobi_hermitian(m, GW, w, Q);
    std::vector<int> order(m);
    for (int i = 0; i < m; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int i, int j) { return w[i] > w[j]; });
    const double mu_max = w[order[0]];
    if (!(mu_max > 0)) return fail(QS_EINVAL, std::string(who) + ": the Kraus step annihilated the state");
    int nz = 0;
    for (int i = 0; i < m; ++i)
        if (w[order[i]] > zero_tol * mu_max) ++nz;
    int keep = std::min(nz, f->r);
    if (nz > f->r)
        while (keep > 0 && w[order[keep - 1]] - w[order[keep]] <= tau * mu_max) --keep;
    if (keep < 1) return fail(QS_EINVAL, std::string(who) + ": tie cluster covers every kept eigenvalue");
    double kept = 0;
    for (int i = 0; i < keep; ++i) kept += w[order[i]];
    const double scale = 1.0 / std::sqrt(kept);
    // coef[(x' * 8 + k'), (y * 8 + c)] = sum_a Q[(a, c), k'] E_a[x'][y] / sqrt(kept)
    double *coef = f->host + kFrHostGram;
    std::memset(coef, 0, (size_t)G * G * 2 * sizeof(double));
    for (int xo = 0; xo < d; ++xo)
        for (int ko = 0; ko < keep; ++ko)
            for (int y = 0; y < d; ++y)
                for (int c = 0; c < rin; ++c) {
                    cd acc = 0;
                    for (int a = 0; a < n_ops; ++a) acc += Q[(size_t)(a * rin + c) * m + order[ko]] * E(a, xo, y);
                    acc *= scale;
                    size_t i = (size_t)(xo * 8 + ko) * G + (y * 8 + c);
                    coef[2 * i] = acc.real();
                    coef[2 * i + 1] = acc.imag();
                }
    double *coef_dev = f->scratch + f->off_coef;
    QS_HIP(hipMemcpyAsync(coef_dev, coef, (size_t)G * G * 2 * sizeof(double), hipMemcpyHostToDevice, f->st));
    if (k == 1) QS_HIP(launch_fr_recombine(f->V, f->dt, f->n, rin, keep, qb[0], coef_dev, f->st));
    else QS_HIP(launch_fr_recombine2(f->V, f->dt, f->n, rin, keep, qb[0], qb[1], coef_dev, f->st));
    // the staging buffer is next written after the next step's synchronisation, which orders it
    // after this upload
    f->rank = keep;
    f->log_trace += std::log(kept);
    if (rank_out) *rank_out = keep;
    return QS_OK;
}

static qs_status fr_check_kraus(qs_fr f, int k, const int32_t *qb, int n_ops, const double *ops, double tau,
                                double zero_tol, const char *who)
{
    if (!f || !ops) return fail(QS_EINVAL, std::string(who) + ": NULL argument");
    if (f->rank < 1) return fail(QS_EINVAL, std::string(who) + ": call fr_init_basis first");
    for (int i = 0; i < k; ++i)
        if (qb[i] < 0 || qb[i] >= f->n) return fail(QS_EINVAL, std::string(who) + ": qubit out of range");
    if (k == 2 && qb[0] == qb[1]) return fail(QS_EINVAL, std::string(who) + ": the two qubits must differ");
    if (n_ops < 1 || n_ops > 4) return fail(QS_EINVAL, std::string(who) + ": n_ops must be in 1..4");
    if (!(tau >= 0) || !(zero_tol >= 0))
        return fail(QS_EINVAL, std::string(who) + ": tau and zero_tol must be >= 0");
    const int words = 2 * (1 << (2 * k)) * n_ops;
    for (int i = 0; i < words; ++i)
        if (!std::isfinite(ops[i])) return fail(QS_EINVAL, std::string(who) + ": non-finite operator entry");
    return QS_OK;
}

// The noisy controlled phase's Kraus pair: eq. (9), or eq. (14) (the same channel, its operators
// mixed by the unitary of eq. (13)), each times the ideal phase diag(1, 1, 1, e^{-i theta}).
// P = exp(-e^2); f = (sqrt(1 + 3P) - 1 - P) / sqrt(P (1 - P)), 0 in the limit P -> 1.
static void kraus_cp_ops(double theta, double e, int improved, double *out)
{
    std::memset(out, 0, 64 * sizeof(double));
    const double P = std::exp(-e * e);
    const cd u11(std::cos(theta), -std::sin(theta));
    auto put = [&](int a, int i, cd v) {
        out[32 * a + 2 * (5 * i)] = v.real();
        out[32 * a + 2 * (5 * i) + 1] = v.imag();
    };
    if (!improved) {
        for (int i = 0; i < 3; ++i) put(0, i, 1.0);
        put(0, 3, u11 * std::sqrt(P));
        put(1, 3, u11 * std::sqrt(1.0 - P));
        return;
    }
    const double f = P >= 1.0 ? 0.0 : (std::sqrt(1.0 + 3.0 * P) - 1.0 - P) / std::sqrt(P * (1.0 - P));
    const double norm = 1.0 / std::sqrt(1.0 + f * f);
    for (int i = 0; i < 3; ++i) {
        put(0, i, norm);
        put(1, i, -f * norm);
    }
    put(0, 3, u11 * ((std::sqrt(P) + f * std::sqrt(1.0 - P)) * norm));
    put(1, 3, u11 * ((std::sqrt(1.0 - P) - f * std::sqrt(P)) * norm));
}

extern "C" {

qs_status qs_kraus_cp(double theta, double e, int improved, double *ops_out)
{
    clear_error();
    if (!ops_out) return fail(QS_EINVAL, "kraus_cp: ops_out is NULL");
    if (!std::isfinite(theta) || !std::isfinite(e) || e < 0)
        return fail(QS_EINVAL, "kraus_cp: theta must be finite and e finite and >= 0");
    if (improved != 0 && improved != 1) return fail(QS_EINVAL, "kraus_cp: improved must be 0 or 1");
    kraus_cp_ops(theta, e, improved, ops_out);
    return QS_OK;
}

qs_status qs_fr_apply_kraus(qs_fr f, int q, int n_ops, const double *ops, double tau, double zero_tol,
                            int *rank_out)
{
    clear_error();
    const int32_t qb[2] = {q, 0};
    qs_status v = fr_check_kraus(f, 1, qb, n_ops, ops, tau, zero_tol, "fr_apply_kraus");
    if (v != QS_OK) return v;
    return fr_kraus_step(f, 1, qb, n_ops, ops, tau, zero_tol, rank_out, "fr_apply_kraus");
}

qs_status qs_fr_apply_kraus2(qs_fr f, int q0, int q1, int n_ops, const double *ops, double tau,
                             double zero_tol, int *rank_out)
{
    clear_error();
    const int32_t qb[2] = {q0, q1};
    qs_status v = fr_check_kraus(f, 2, qb, n_ops, ops, tau, zero_tol, "fr_apply_kraus2");
    if (v != QS_OK) return v;
    return fr_kraus_step(f, 2, qb, n_ops, ops, tau, zero_tol, rank_out, "fr_apply_kraus2");
}

qs_status qs_fr_apply_noisy_gate(qs_fr f, const qs_gate *g, double e, double tau, double zero_tol,
                                 int *rank_out)
{
    clear_error();
    if (!f || !g) return fail(QS_EINVAL, "fr_apply_noisy_gate: NULL argument");
    if (!std::isfinite(e) || e < 0) return fail(QS_EINVAL, "fr_apply_noisy_gate: e must be finite and >= 0");
    qs_status v = check_gate(*g, f->n, 0);
    if (v != QS_OK) return v;
    if (g->kind == QS_G_U1 && e > 0 && g->noise == QS_NOISE_ROT) {
        double ops[16];
        kraus_rot_ops(g->m, e, ops);
        return qs_fr_apply_kraus(f, g->q0, 2, ops, tau, zero_tol, rank_out);
    }
    if (g->kind == QS_G_CP && e > 0 && g->noise == QS_NOISE_PHASE) {
        double ops[64];
        kraus_cp_ops(g->theta, e, 0, ops);
        return qs_fr_apply_kraus2(f, g->q0, g->q1, 2, ops, tau, zero_tol, rank_out);
    }
    v = qs_fr_apply_gate(f, g);
    if (v == QS_OK && rank_out) *rank_out = f->rank;
    return v;
}

qs_status qs_fr_fidelity(qs_fr f, qs_state psi, int tpsi, double *f_unnorm, double *f_norm, double *log_trace)
{
    clear_error();
    if (!f || !psi) return fail(QS_EINVAL, "fr_fidelity: NULL argument");
    if (psi->n != f->n || psi->dt != f->dt) return fail(QS_EINVAL, "fr_fidelity: psi differs in n or dtype");
    if (tpsi < 0 || tpsi >= psi->T) return fail(QS_EINVAL, "fr_fidelity: trajectory out of range");
    if (f->rank < 1) return fail(QS_EINVAL, "fr_fidelity: call fr_init_basis first");
    const char *pp = (const char *)psi->buf + (amp_bytes(psi->dt) << psi->n) * tpsi;
    if (psi->st != f->st) QS_HIP(hipStreamSynchronize(psi->st));
    double *out = f->scratch + f->off_ovo;
    QS_HIP(launch_overlaps(pp, 0, f->V, f->dt, f->n, f->rank, -1, f->scratch + f->off_ovp, out, f->st));
    double h[40];
    QS_HIP(hipMemcpyAsync(h, out, sizeof(double) * 5 * f->rank, hipMemcpyDeviceToHost, f->st));
    QS_HIP(hipStreamSynchronize(f->st));
    double s = 0;
    for (int c = 0; c < f->rank; ++c) s += h[5 * c] * h[5 * c] + h[5 * c + 1] * h[5 * c + 1];
    if (f_norm) *f_norm = s;
    if (f_unnorm) *f_unnorm = s * std::exp(f->log_trace);
    if (log_trace) *log_trace = f->log_trace;
    return QS_OK;
}

qs_status qs_fr_info(qs_fr f, int *rank, double *log_trace, void **columns_dev)
{
    clear_error();
    if (!f) return fail(QS_EINVAL, "fr_info: NULL handle");
    if (rank) *rank = f->rank;
    if (log_trace) *log_trace = f->log_trace;
    if (columns_dev) *columns_dev = f->V;
    return QS_OK;
}

}  // extern "C"
