// Internal declarations shared by the host runtime and the gfx950 kernels of libqsim.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "qsim.h"

namespace qs {

// ---------------------------------------------------------------------------------------
// Errors: every C entry point returns a qs_status and leaves a thread-local message.
// ---------------------------------------------------------------------------------------
qs_status fail(qs_status st, const std::string &msg);
qs_status hip_fail(hipError_t e, const char *what);
void clear_error();

#define QS_HIP(call)                                   \
    do {                                               \
        hipError_t _e = (call);                        \
        if (_e != hipSuccess) return qs::hip_fail(_e, #call); \
    } while (0)

// ---------------------------------------------------------------------------------------
// Fused-pass program (device side).  A pass loads tiles of 2^K amplitudes whose tile-local
// index bit j is physical index bit q_pos[j]; the remaining n - K bits enumerate tiles.  Each
// thread holds 2^RB amplitudes in registers; a round fixes which RB tile-local bits are the
// register bits (reg_mask) and applies its ops in registers; rounds are linked by exchanges
// through LDS.  Tile-local bits not in reg_mask are the thread-id bits in increasing order.
// ---------------------------------------------------------------------------------------
constexpr int kMaxTileBits = 15;
constexpr int kMaxRegBits = 4;

struct PassDesc {
    int32_t K;
    int32_t RB;
    int32_t round_begin;
    int32_t round_end;
    uint64_t outer_mask;          // physical bits (< n) that are not in the tile
    int32_t q_pos[16];            // tile-local bit j -> physical bit
};

struct RoundDesc {
    uint32_t reg_mask;            // tile-local bits held in registers during this round
    int32_t op_begin;
    int32_t op_end;
    int32_t reserved;
};

enum OpType : int32_t { OP_U1 = 0, OP_U2 = 1, OP_DIAG = 2 };
enum DiagKind : int32_t { DIAG_NEGATE = 0, DIAG_PHASE = 1 };
enum PhaseClass : int32_t { PH_OUTER = 0, PH_THREAD = 1, PH_REG = 2 };

struct OpDesc {
    int32_t type;
    int32_t p0, p1;               // register-bit positions of the target(s)
    int32_t gate;                 // gate index: noise-table row / matrix of the gate
    int32_t pre_begin, pre_end;   // PhaseRefs applied to the |1> input of a U1 (column phases)
    int32_t post_begin, post_end; // PhaseRefs applied to the |1> output of a U1 (row phases)
    int32_t diag_kind;
    uint32_t lmask, lvalue;       // DIAG: tile-local condition (l & lmask) == lvalue
    uint32_t reserved;
    uint64_t omask, ovalue;       // DIAG: tile condition (outer index & omask) == ovalue
};

// A controlled phase folded into a U1: multiply by the phase of gate `gate` when the
// condition bit is 1.  cls PH_OUTER: physical bit `bit` of the tile's outer index;
// PH_THREAD: tile-local bit `bit` of the thread's base index; PH_REG: register bit `bit`.
struct PhaseRef {
    int32_t cls;
    int32_t bit;
    int32_t gate;
    int32_t reserved;
};

// ---------------------------------------------------------------------------------------
// Launchers (kernels.hip / fused.hip / fr.hip).  All asynchronous on `st`.
// Noise table: tab[(g * S + s) * 8 + 0..7] = complex 2x2 (U1) or phase in [0..1] (CP), FP64.
// ---------------------------------------------------------------------------------------
struct NoiseArgs {
    double e;                     // used when e_dev == nullptr
    const double *e_dev;          // per-slot strength (device, S entries) or nullptr
    uint64_t seed;
    uint32_t request;
    uint32_t traj_base;           // counter of slot first_noisy_slot
    int32_t first_noisy_slot;     // slots below this one are ideal (e = 0)
};

hipError_t launch_noise_table(const qs_gate *gates_dev, int n_gates, int S, NoiseArgs na,
                              double *tab, hipStream_t st);
hipError_t launch_noise_draw(uint64_t seed, uint32_t request, uint32_t stream,
                             const uint32_t *sites, int n_sites, uint32_t traj_base, int n_traj,
                             double *out, hipStream_t st);
hipError_t launch_init_basis(void *psi, qs_dtype dt, int n, int S, uint64_t index, hipStream_t st);
hipError_t launch_sweep_u1(void *psi, qs_dtype dt, int n, int S, int q, const double *tab_row,
                           hipStream_t st);
hipError_t launch_sweep_cp(void *psi, qs_dtype dt, int n, int S, int qa, int qb,
                           const double *tab_row, hipStream_t st);
hipError_t launch_sweep_perm(void *psi, qs_dtype dt, int n, int S, int kind, int qa, int qb,
                             hipStream_t st);
// m32: host 4x4 complex matrix (32 doubles), passed to the kernel by value.
hipError_t launch_sweep_2q(void *psi, qs_dtype dt, int n, int S, int qa, int qb,
                           const double *m32, hipStream_t st);
// One gate's operator for S slots (as launch_noise_table for a single gate passed by value).
hipError_t launch_noise_one(const qs_gate &g, int S, NoiseArgs na, double *tab, hipStream_t st);
hipError_t launch_flip(void *psi, qs_dtype dt, int n, int S, uint64_t mask, uint64_t value,
                       hipStream_t st);
// Per-slot (Re <ref|psi_s>, Im <ref|psi_s>, <psi_s|psi_s>, Re psi_s[marked], Im psi_s[marked])
// with ref = slot ref_slot of ref_psi; out has S * 5 doubles.  partials: reduce_partials_size.
size_t reduce_partials_doubles(int n, int S);
hipError_t launch_overlaps(const void *ref_psi, int ref_slot, const void *psi, qs_dtype dt, int n,
                           int S, int64_t marked, double *partials, double *out, hipStream_t st);
// <psi|rho|psi> and Tr rho over vec(rho) of n qubits: out = (Re f, Im f, Re tr, Im tr).
hipError_t launch_dm_expect(const void *rho, const void *psi, qs_dtype dt, int n,
                            double *partials, double *out, hipStream_t st);
hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t st);

hipError_t launch_fused_pass(void *psi, qs_dtype dt, int n, int S, const PassDesc *pass_host,
                             const PassDesc *pass_dev, const RoundDesc *rounds,
                             const OpDesc *ops, const PhaseRef *prefs, const double *tab,
                             const qs_gate *gates_dev, hipStream_t st);
size_t fused_lds_bytes(qs_dtype dt, int K);

// Fixed rank: Gram of the 2r half-columns; partial blocks then a fixed-order final sum.
size_t fr_gram_partials_doubles(int n, int r);
hipError_t launch_fr_gram(const void *V, qs_dtype dt, int n, int r, int q, double *partials,
                          double *gram_out, hipStream_t st);
hipError_t launch_fr_recombine(void *V, qs_dtype dt, int n, int r_in, int r_out, int q,
                               const double *coef_dev, hipStream_t st);

// ---------------------------------------------------------------------------------------
// Kernel timing (HIP events around each launch while enabled).
// ---------------------------------------------------------------------------------------
struct TimedLaunch {
    const char *name;
    double alg_bytes;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    bool on = false;
    TimedLaunch(const char *nm, double bytes, hipStream_t s);
    ~TimedLaunch();
};

// ---------------------------------------------------------------------------------------
// Fusion planner (planner.cpp).
// ---------------------------------------------------------------------------------------
struct Program {
    std::vector<PassDesc> passes;
    std::vector<RoundDesc> rounds;
    std::vector<OpDesc> ops;
    std::vector<PhaseRef> prefs;
    std::vector<int32_t> layout;  // logical qubit -> physical bit after the circuit
    int K = 0, RB = 0;
};

qs_status plan_fused(const qs_gate *gates, int n_gates, int n, int K, int RB, int run_bits,
                     Program &out);

inline size_t amp_bytes(qs_dtype dt) { return dt == QS_C64 ? 8 : 16; }
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace qs
