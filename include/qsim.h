/*
 * qsim.h -- C ABI of the MI355X (gfx950) noisy quantum-circuit library.
 *
 * The method is that of Bogdanov, Chernyavskiy et al., "Numerical and analytical research of
 * the impact of decoherence on quantum circuits" (arXiv:1412.2293):
 *   - Section 2: a circuit is the product U_s ... U_1 |psi0>; a one-qubit gate updates every
 *     amplitude pair that differs only in the target bit; Monte Carlo noise replaces a
 *     one-qubit gate U by U * V(e*xi) (eq. 1) and a controlled phase theta by theta + e*xi
 *     (eq. 2 and the sentence after it), xi ~ N(0,1).
 *   - Section 3: rho as the vector sum rho_ij |i>|j>, gates as U (x) U*, noise as Kraus sums
 *     sum_k E_k rho E_k^dagger (eq. 3), Kraus sets of eq. (6) and eq. (9).
 *   - Section 3.2: the fixed-rank approximation of rho, truncated by spectral decomposition
 *     after every noisy step and renormalised.
 *
 * Conventions for every entry point:
 *   - Qubit q is bit q of the amplitude index (qubit 0 is the least significant bit).
 *   - A state buffer holds n_traj state vectors one after the other, each 2^n complex
 *     amplitudes, interleaved (re, im), in float (QS_C64) or double (QS_C128).
 *   - A density matrix of n qubits is a state of 2n qubits holding vec(rho), entry rho_ij at
 *     index i * 2^n + j (ket bits high, bra bits low).
 *   - Device buffers are BORROWED: the caller allocates them (for example as torch tensors),
 *     keeps them alive while the library uses them and frees them; the library never frees
 *     a caller buffer.  Handles own only their metadata and small device scratch that the
 *     matching *_destroy frees.
 *   - Streams are the caller's (hipStream_t passed as void*; NULL = the default stream).
 *     Calls enqueue asynchronously on the handle's stream unless they return host values
 *     (fidelities, ranks), which synchronise that stream before returning.
 *   - Every call validates all arguments before enqueueing anything: on error nothing has
 *     been enqueued, the call returns a negative qs_status and qs_last_error() (thread-local)
 *     describes the problem.  Nothing throws or aborts across this boundary.
 *   - One host thread per handle at a time.  Indices are 64-bit.
 *   - Results depend only on the circuit, the seed, the request id, the trajectory counter,
 *     the dtype and the plan; not on batch composition or timing.
 */
#ifndef QSIM_H
#define QSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QS_OK = 0,
    QS_EINVAL = -1,       /* invalid argument (range, size, null pointer, buffer too small) */
    QS_ENOMEM = -2,       /* the library could not allocate its own small scratch            */
    QS_EDEVICE = -3,      /* a HIP runtime call failed                                       */
    QS_EUNSUPPORTED = -4, /* valid request this build does not implement                     */
    QS_EBUSY = -5         /* serving: admission refused (no free memory or slot)             */
} qs_status;

/* Amplitude type.  The two range markers make every 32-bit int a value of the type, so a
 * caller's out-of-range value reaches the library's validation (QS_EINVAL, or 0 bytes) as a
 * well-defined value; they are not valid arguments. */
typedef enum {
    QS_C64 = 0,
    QS_C128 = 1,
    QS_DTYPE_RANGE_MIN_ = -0x7fffffff - 1,
    QS_DTYPE_RANGE_MAX_ = 0x7fffffff
} qs_dtype;

/* Gate kinds. */
typedef enum {
    QS_G_U1 = 0,   /* dense one-qubit gate m (2x2) on q0                                    */
    QS_G_CP = 1,   /* controlled phase, eq. (2): |11> of (q0, q1) times exp(-i theta); CZ = pi */
    QS_G_SWAP = 2, /* exchange qubits q0, q1                                                  */
    QS_G_CNOT = 3, /* control q0, target q1                                                   */
    QS_G_U2 = 4,   /* dense two-qubit gate m (4x4), local index bit(q0) + 2 bit(q1)           */
    QS_G_FLIP = 5, /* negate every amplitude i with (i & mask) == value                       */
    QS_G_DIAG = 6  /* multiply every amplitude i with (i & mask) == value by the complex factor
                      m[0] + i m[1] (a diagonal gate on the masked bits: a sign flip, a
                      controlled phase with any number of controls, or one of the non-unitary
                      diagonal factors of an averaged channel on vec(rho)); noiseless          */
} qs_gate_kind;

/* Noise tags (Section 2). */
typedef enum {
    QS_NOISE_NONE = 0,
    QS_NOISE_ROT = 1,   /* one-qubit gate U becomes U * V(e xi), V = [[c, s], [-s, c]], eq. (1) */
    QS_NOISE_PHASE = 2  /* controlled phase theta becomes theta + e xi                         */
} qs_noise_kind;

/* One gate.  m holds a row-major complex matrix, (re, im) interleaved: 2x2 in m[0..7] for
 * U1, 4x4 in m[0..31] for U2; unused otherwise.  `site` is the first Philox counter word of
 * this gate's noise draw (normally the gate's position in its circuit). */
typedef struct {
    int32_t kind;
    int32_t q0;
    int32_t q1;
    int32_t noise;
    uint32_t site;
    uint32_t reserved;
    double theta;
    uint64_t mask;
    uint64_t value;
    double m[32];
} qs_gate;

/* Noise parameters.  Trajectory t of a batch draws xi from Philox4x32-10 with counter
 * (site, traj_base + t, 0, request) and key (seed & 0xffffffff, seed >> 32); the two first
 * words give u1 = (top 53 bits + 1) 2^-53, the two last u2 = (top 53 bits) 2^-53 and
 * xi = sqrt(-2 ln u1) cos(2 pi u2).  e_per_traj (host array, n_traj entries) overrides e. */
typedef struct {
    double e;
    uint64_t seed;
    uint32_t request;
    uint32_t traj_base;
    const double *e_per_traj;
} qs_noise;

/* Execution plan for run_trajectories. */
typedef struct {
    int32_t fuse;      /* 0: one sweep kernel per gate; 1: fused passes; -1: library picks
                          (qs_plan_choose) unless a tile shape is given, then fused        */
    int32_t tile_bits; /* fused: amplitudes per tile = 2^tile_bits (0 = library picks)      */
    int32_t reg_bits;  /* fused: amplitudes per thread = 2^reg_bits (0 = library picks)     */
    int32_t run_bits;  /* fused: the 2^run_bits lowest-index amplitudes of a tile are one
                          contiguous row (coalescing); 0 = library picks                   */
    int32_t mfma;      /* fused, complex<float>, 4 register bits: 1 runs each register round of
                          three or more one-qubit ops as one dense 16 x 16 complex block (the
                          ops and their phases conditioned on register bits multiplied
                          together) on the FP32 matrix cores, as a real 32 x 32 product;
                          0 = op by op on the vector ALUs.  Ignored otherwise.              */
} qs_plan;

typedef struct qs_state_s *qs_state;
typedef struct qs_fr_s *qs_fr;

/* Thread-local description of the last error (empty string if none). */
const char *qs_last_error(void);
const char *qs_version(void);

/* ------------------------------------------------------------------------------------------
 * State vectors (Section 2).
 * ---------------------------------------------------------------------------------------- */

/* Bytes of a buffer holding n_traj states of n qubits (n in 1..34). */
size_t qs_sv_bytes_required(int n_qubits, qs_dtype dt, int n_traj);

/* Wrap a caller buffer (>= qs_sv_bytes_required bytes, 256-byte aligned device memory) as
 * n_traj state vectors of n qubits.  The contents are left as they are. */
qs_status qs_sv_create(int n_qubits, qs_dtype dt, int n_traj, void *dev_buf, size_t buf_bytes,
                       void *hip_stream, qs_state *out);
qs_status qs_sv_destroy(qs_state s);

/* Every trajectory <- the basis state |index>. */
qs_status qs_sv_init_basis(qs_state s, uint64_t index);

/* Apply one gate to every trajectory of s as one sweep over the state buffer (Section 2:
 * the amplitude-pair update of a one-qubit gate, its 4-tuple analogue for two qubits).
 * nz == NULL or nz->e == 0 applies the ideal gate; otherwise trajectory t is noisy with the
 * counter of qs_noise (nz->e_per_traj must be NULL here; run_trajectories takes it).
 * Qubits must be distinct and < n.  Asynchronous. */
qs_status qs_apply_gate(qs_state s, const qs_gate *g, const qs_noise *nz);

/* Kraus channel on vec(rho) (eq. 3), asynchronous: rho <- sum_k E_k rho E_k^dagger.  `rho` is a state of 2n
 * qubits (n_traj == 1) holding vec(rho) of an n-qubit density matrix; k = 1 or 2 target
 * qubits `qubits` (< n); ops: n_ops host matrices of 2^k x 2^k complex doubles, row-major,
 * (re, im) interleaved, local index bit(qubits[0]) + 2 bit(qubits[1]).  The library forms the
 * superoperator sum_k E_k (x) conj(E_k) in FP64 and applies it in one sweep over the ket
 * bits qubits + n and the bra bits qubits (k = 2: a 16 x 16 update on four index bits, the
 * superoperator uploaded through a pinned buffer of the handle; a call waits until the previous
 * k = 2 call's upload has left that buffer).  Errors: k other than 1, 2 (QS_EUNSUPPORTED);
 * qubits out of range or equal, n_ops outside 1..64, non-finite entries (QS_EINVAL). */
qs_status qs_apply_kraus(qs_state rho, int k, const int32_t *qubits, int n_ops, const double *ops);

/* One circuit gate on vec(rho) (Section 3): a ROT-tagged one-qubit gate U with e > 0 becomes
 * its Kraus channel {U E1, U E2} with E1, E2 of eq. (6) (lambda_1,2 = (1 +- exp(-2 e^2)) / 2),
 * applied as one superoperator sweep; other one-qubit gates as U (x) U*; SWAP, CNOT, U2 and
 * noiseless CP as U on the ket bits then U* on the bra bits; FLIP as the sign flip of the
 * selected rows and columns.  A PHASE-tagged CP with e > 0 becomes its averaged channel
 * (eq. 9): entry rho_ij is multiplied by exp(-i theta (b_i - b_j)) exp(-e^2 (b_i - b_j)^2 / 2)
 * where b = 1 when both qubits of the row (column) index are 1.
 * Asynchronous. */
qs_status qs_dm_apply_gate(qs_state rho, const qs_gate *g, double e);

/* Kraus pair of the noisy controlled phase theta with phase-noise strength e (Section 3.3),
 * each operator times the ideal gate diag(1, 1, 1, exp(-i theta)), written to ops_out as two
 * 4x4 complex matrices (64 doubles, row-major, (re, im) interleaved, local index
 * bit(q0) + 2 bit(q1); the operators are diagonal).  With P = exp(-e^2):
 *   improved = 0: eq. (9), E1 = diag(1, 1, 1, sqrt(P)), E2 = diag(0, 0, 0, sqrt(1 - P));
 *   improved = 1: eq. (14), the eq. (9) pair mixed by the unitary of eq. (13) with
 *     f = (sqrt(1 + 3P) - 1 - P) / sqrt(P (1 - P)) (0 at P = 1):
 *     E1 = diag(1, 1, 1, sqrt(P) + f sqrt(1 - P)) / sqrt(1 + f^2),
 *     E2 = diag(-f, -f, -f, sqrt(1 - P) - f sqrt(P)) / sqrt(1 + f^2).
 * Both describe the same channel.  Errors: NULL ops_out, non-finite theta or e, e < 0, improved
 * other than 0 or 1 (QS_EINVAL).  Host only, no device work. */
qs_status qs_kraus_cp(double theta, double e, int improved, double *ops_out);

/* F = |<a_ta|b_tb>|^2 / (<a|a><b|b>) in FP64 (Section 2, Fig. 1 uses 1 - F); both states must
 * have the same n and dtype.  overlap (nullable) receives <a|b> as two doubles.  Blocks. */
qs_status qs_fidelity(qs_state a, int ta, qs_state b, int tb, double *f, double *overlap);

/* Allocation-free form of qs_fidelity's reductions, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * no handle, no hipMalloc or hipFree, no allocating library call.  a_dev and b_dev are two
 * caller-owned device state vectors of n_qubits (1..34) qubits in dtype dt; out_dev (device,
 * 4 doubles, caller-owned) receives Re <a|b>, Im <a|b>, <a|a>, <b|b> in FP64, the same sums in the
 * same order as qs_fidelity (F = |<a|b>|^2 / (<a|a> <b|b>)).  The partial sums live in a fixed
 * 16.1 KiB device array of the library (one copy per GPU, held until the process ends); a call
 * enqueues on hip_stream and returns without waiting.  Calls that overlap on one GPU (other
 * streams or host threads) race on that array; calls on one stream are ordered.  Errors:
 * NULL pointers, unknown dtype, n_qubits outside 1..34 (QS_EINVAL), a failed HIP call
 * (QS_EDEVICE). */
qs_status qs_fidelity_noalloc(const void *a_dev, const void *b_dev, int n_qubits, qs_dtype dt,
                              void *hip_stream, double *out_dev);

/* <psi|rho|psi> = sum_ij conj(psi_i) rho_ij psi_j and Tr rho, FP64 (Section 3).  rho as in
 * qs_apply_kraus, psi trajectory tpsi of an n-qubit state of the same dtype.  Blocks. */
qs_status qs_dm_fidelity(qs_state rho, qs_state psi, int tpsi, double *f, double *trace);

/* ------------------------------------------------------------------------------------------
 * Density-matrix circuit runs (Section 3) through the fused passes: the noisy n-qubit circuit
 * becomes a noiseless circuit on vec(rho) (2n qubits, entry rho_ij at index i 2^n + j), which
 * the trajectory machinery runs as one slot, tile by tile, many channels per pass.
 * ---------------------------------------------------------------------------------------- */

/* The superoperator circuit of gates with noise strength e, written to out (host, cap
 * entries; out NULL: only *n_out is set).  Every output gate is noiseless:
 *   - ROT-tagged one-qubit U with e > 0: its eq. (6) Kraus pair {U E1, U E2} as one U2 gate on
 *     (q0 = q, q1 = q + n) with m[b + 2a][b' + 2a'] = sum_k K_k[a][a'] conj(K_k[b][b'])
 *     (a, a': row bit; b, b': column bit);
 *   - PHASE-tagged CP with e > 0: its eq. (9) average as three DIAG gates, rows with both
 *     qubits 1 by exp(-i theta) exp(-e^2/2), columns with both by exp(i theta) exp(-e^2/2),
 *     entries with all four by exp(e^2);
 *   - any other gate G: G on the row bits (qubits + n, masks << n), then conj(G) on the column
 *     bits (CP with -theta, U1/U2/DIAG with conjugated entries).
 * Errors: n_qubits outside 1..17, e < 0 or not finite, an invalid gate, cap too small
 * (QS_EINVAL).  Host only. */
qs_status qs_dm_superop(const qs_gate *gates, int n_gates, int n_qubits, double e, qs_gate *out, int cap,
                        int *n_out);

/* Bytes of dev_buf needed by qs_dm_run (0 on invalid arguments). */
size_t qs_dm_run_bytes_required(const qs_gate *gates, int n_gates, int n_qubits, qs_dtype dt, double e,
                                const qs_plan *plan);

/* rho = the channel of the noisy circuit applied to |init><init| (Section 3: ROT noise as the
 * eq. (6) Kraus pair, PHASE noise as the eq. (9) average), computed by running the
 * qs_dm_superop circuit under `plan` (as in qs_run_trajectories: fused passes or per-gate
 * sweeps, chosen by the library for fuse = -1).  f_out (host) = <psi|rho|psi> =
 * sum_ij conj(psi_i) rho_ij psi_j and trace_out (host, nullable) = Tr rho, in FP64, with psi_dev
 * a caller-owned device state of n_qubits qubits in dtype dt and logical qubit order (the ideal
 * state, normally).  vec(rho) stays in dev_buf at byte offset 0 with row bit q at physical bit
 * layout_out[q] + n and column bit q at layout_out[q] (layout_out: nullable, n entries;
 * SWAPs relabel both halves alike).  Blocks until the results are on the host.  Errors as
 * qs_dm_superop, plus init_index out of range, NULL psi_dev or f_out, an unaligned or small
 * buffer (QS_EINVAL), a failed HIP call (QS_EDEVICE). */
qs_status qs_dm_run(const qs_gate *gates, int n_gates, int n_qubits, uint64_t init_index, qs_dtype dt, double e,
                    const qs_plan *plan, const void *psi_dev, void *dev_buf, size_t buf_bytes, void *hip_stream,
                    double *f_out, double *trace_out, int32_t *layout_out);

/* Device noise draws for testing: out_dev[t * n_sites + s] = xi for (sites_dev[s],
 * traj_base + t) on Philox stream `stream` (FP64, device memory).  Asynchronous. */
qs_status qs_noise_draw(uint64_t seed, uint32_t request, uint32_t stream,
                        const uint32_t *sites_dev, int n_sites, uint32_t traj_base, int n_traj,
                        double *out_dev, void *hip_stream);

/* ------------------------------------------------------------------------------------------
 * Monte Carlo trajectories (Section 2, Fig. 1): the ideal circuit and n_traj noisy copies,
 * run as one batch, with the fidelity of each noisy state to the ideal one.
 * ---------------------------------------------------------------------------------------- */

/* Bytes of dev_buf needed by qs_run_trajectories for this circuit and plan; 0 on a rejected
 * argument (qs_last_error says which).  Plans the circuit as qs_run_trajectories does and keeps
 * the result in the library's small cache of recent circuits, so the run that follows (or a
 * repeated query) does not plan again.  No device work. */
size_t qs_traj_bytes_required(const qs_gate *gates, int n_gates, int n_qubits, qs_dtype dt,
                              int n_traj, const qs_plan *plan);

/* Run the circuit from |init_index> on n_traj + 1 states held in dev_buf: slot 0 is the ideal
 * circuit, slot t + 1 trajectory t.  fid_out[t] (host, FP64) = |<ideal|psi_t>|^2 /
 * (<ideal|ideal><psi_t|psi_t>); p_out[t] (nullable) = |psi_t[marked]|^2 when marked >= 0;
 * norm_out[t] (nullable) = <psi_t|psi_t>.  The final states stay in dev_buf (slot s at byte
 * offset s * 2^n * amplitude size), in the physical qubit order layout_out[q] (nullable,
 * n entries): logical qubit q sits at bit layout_out[q] (fused plans turn SWAP gates into a
 * relabelling instead of moving data).  Blocks until the results are on the host. */
qs_status qs_run_trajectories(const qs_gate *gates, int n_gates, int n_qubits,
                              uint64_t init_index, qs_dtype dt, const qs_noise *nz, int n_traj,
                              int64_t marked, const qs_plan *plan, void *dev_buf,
                              size_t buf_bytes, void *hip_stream, double *fid_out,
                              double *p_out, double *norm_out, int32_t *layout_out);

/* Captured trajectory runs: the whole launch sequence of qs_run_trajectories for one circuit,
 * n_traj and buffer, recorded once as a HIP graph and replayed per run.  The per-run values
 * (noise seed, request, trajectory base, per-trajectory strengths, initial and marked index)
 * travel through pinned host memory and device memory read by the kernels, so one graph
 * serves every run; results equal qs_run_trajectories with the same plan bit for bit.  For
 * circuits whose passes are short (small n, many gates) replay removes the per-launch host
 * cost.  The graph owns a stream, pinned buffers and the instantiated graph; the caller owns
 * dev_buf, which must stay allocated and unused by other work until qs_traj_graph_destroy. */
typedef struct qs_traj_graph_s *qs_traj_graph;
qs_status qs_traj_graph_bytes_required(const qs_gate *gates, int n_gates, int n_qubits, qs_dtype dt,
                                       int n_traj, const qs_plan *plan, size_t *bytes);
qs_status qs_traj_graph_create(const qs_gate *gates, int n_gates, int n_qubits, qs_dtype dt, int n_traj,
                               const qs_plan *plan, void *dev_buf, size_t buf_bytes, qs_traj_graph *out);
/* One replay; blocks until the results (as in qs_run_trajectories) are on the host. */
qs_status qs_traj_graph_launch(qs_traj_graph g, uint64_t init_index, const qs_noise *nz, int64_t marked,
                               double *fid_out, double *p_out, double *norm_out, int32_t *layout_out);
qs_status qs_traj_graph_destroy(qs_traj_graph g);

/* Byte offsets, inside the qs_run_trajectories buffer, of its regions (for inspection):
 * out[0] states, [1] noise table (per gate and slot: 8 doubles), [2] device gates, [3] per-slot
 * noise strengths, [4] pass, [5] stage, [6] round, [7] op, [8] phase-reference, [9] outer-job,
 * [10] outer-bit descriptors, [11] phase chains, [12] per-tile tables of the last pass (the
 * tiles' index bits, then the phase products of its outer jobs), [13] per-slot records of the
 * last pass, [14] reduction partials, [15] results, [16] total (out holds 17 values).  No
 * device work. */
qs_status qs_traj_layout(const qs_gate *gates, int n_gates, int n_qubits, qs_dtype dt, int n_traj,
                         const qs_plan *plan, size_t *out);

/* The plan chosen for fuse = -1 (with no tile shape given): unfused sweeps or a fused shape
 * (tile_bits, reg_bits, run_bits) from a fixed set of candidates, whichever a cost model rates
 * fastest for a batch of 64 slots.  The model prices each fused pass at the larger of its
 * HBM time (one read and one write of the state) and its vector-ALU time (per-amplitude
 * instruction counts of its ops), plus launches; unfused runs at each gate's sweep.  The
 * choice depends only on the gates, n and dtype.  *model_s_per_slot (nullable) receives the
 * modelled seconds per state slot.  No device work. */
qs_status qs_plan_choose(const qs_gate *gates, int n_gates, int n_qubits, qs_dtype dt, qs_plan *out,
                         double *model_s_per_slot);

/* The fused-pass program the library builds for this circuit and plan, as JSON text (passes,
 * tile qubits, stages, register rounds, ops with their folded phases, final qubit layout), for
 * inspection and host-side checks.  Writes at most cap bytes including the terminating NUL and
 * returns the full length (excluding NUL) in *len.  No device work. */
qs_status qs_plan_describe(const qs_gate *gates, int n_gates, int n_qubits, qs_dtype dt,
                           const qs_plan *plan, char *buf, size_t cap, size_t *len);

/* Per-kernel timing of the calling thread's launches, measured with HIP events on the stream
 * each kernel is launched on.  While enabled, every launch is bracketed by two events;
 * qs_timing_read synchronises and returns, for kernel class `name` ("sweep_u1", "sweep_cp",
 * "sweep_swap", "sweep_2q", "flip", "fused", "reduce", "noise", "init", "fr_gram",
 * "fr_recombine", "copy"), the number of launches, their summed duration in ms and their
 * summed algorithmic bytes (what the method must move: read + write of the touched
 * amplitudes). */
qs_status qs_timing_enable(int on);
qs_status qs_timing_read(const char *name, int64_t *launches, double *ms, double *alg_bytes);
qs_status qs_timing_reset(void);

/* Plain device copy of `bytes` (multiple of 16) from src to dst, for bandwidth calibration. */
qs_status qs_copy(void *dst, const void *src, size_t bytes, void *hip_stream);

/* ------------------------------------------------------------------------------------------
 * Fixed-rank density matrix (Section 3.2): rho = exp(log_trace) sum_{j<rank} |v_j><v_j|,
 * columns v_j stored as `r` state vectors of n qubits, orthogonal, sum <v_j|v_j> = 1.
 * ---------------------------------------------------------------------------------------- */
size_t qs_fr_bytes_required(int n_qubits, int r, qs_dtype dt);
qs_status qs_fr_create(int n_qubits, int r, qs_dtype dt, void *dev_buf, size_t buf_bytes,
                       void *hip_stream, qs_fr *out);
qs_status qs_fr_destroy(qs_fr fr);
/* rho <- |index><index| (rank 1, log_trace 0). */
qs_status qs_fr_init_basis(qs_fr fr, uint64_t index);
/* A unitary gate (noise ignored) on every column; never truncates. */
qs_status qs_fr_apply_gate(qs_fr fr, const qs_gate *g);
/* One-qubit Kraus set (n_ops <= 4 host 2x2 complex matrices as in qs_apply_kraus) on qubit q:
 * W = [E_k v_j], Gram G = W^dagger W (FP64, one pass over the columns), eigen-decomposition
 * of G in FP64, keep the leading eigenvectors (at most r; eigenvalues <= zero_tol * max are
 * dropped; if the r-th and (r+1)-th are within tau * max the whole tied cluster at the cut is
 * dropped), columns <- W Q / sqrt(kept trace), log_trace += ln(kept trace).  rank_out gets
 * the new rank.  Blocks (the eigen-decomposition runs on the host). */
qs_status qs_fr_apply_kraus(qs_fr fr, int q, int n_ops, const double *ops, double tau,
                            double zero_tol, int *rank_out);
/* Two-qubit Kraus set (Section 3.2 with the two-qubit channels of Section 3.3, eq. 9 and
 * eq. 14): n_ops <= 4 host 4x4 complex matrices, row-major, (re, im) interleaved, local index
 * bit(q0) + 2 bit(q1), on the distinct qubits q0, q1.  The same step as qs_fr_apply_kraus over
 * the 4r quarter-columns of the columns (Gram 32 x 32 in FP64, one read of the columns; the
 * recombination in one read and one write).  Errors as qs_fr_apply_kraus; q0 == q1 is
 * QS_EINVAL.  Blocks. */
qs_status qs_fr_apply_kraus2(qs_fr fr, int q0, int q1, int n_ops, const double *ops, double tau,
                             double zero_tol, int *rank_out);
/* One circuit gate in the fixed-rank form: a ROT-tagged one-qubit gate U with e > 0 is the
 * Kraus step of qs_fr_apply_kraus with {U E1, U E2} of eq. (6); a PHASE-tagged controlled
 * phase with e > 0 is the two-qubit Kraus step of qs_fr_apply_kraus2 with the eq. (9) pair of
 * qs_kraus_cp (improved = 0); any other gate (noise ignored) is qs_fr_apply_gate.  rank_out
 * (nullable) gets the rank afterwards. */
qs_status qs_fr_apply_noisy_gate(qs_fr fr, const qs_gate *g, double e, double tau,
                                 double zero_tol, int *rank_out);
/* <psi|rho|psi>: f_unnorm = exp(log_trace) f_norm, f_norm with the stored unit-trace rho. */
qs_status qs_fr_fidelity(qs_fr fr, qs_state psi, int tpsi, double *f_unnorm, double *f_norm,
                         double *log_trace);
/* Current rank; columns (device pointer of column 0, columns 2^n amplitudes apart). */
qs_status qs_fr_info(qs_fr fr, int *rank, double *log_trace, void **columns_dev);

/* ------------------------------------------------------------------------------------------
 * Request server: continuous batching of Monte Carlo trajectory requests (Section 2's method,
 * run for many independent circuits) on one GPU.  Not described in the paper; a serving form
 * of qs_run_trajectories.
 *
 * The caller hands over one device pool (never freed by the library).  A request is validated
 * and planned in qs_srv_submit, then cut into trajectory batches of one size (at most
 * max_chunk_traj, halved until one batch fits the pool).  A worker thread admits batches in
 * arrival order whenever one of max_inflight streams is idle and the pool has a free range
 * large enough for the batch (first fit, 256-byte granules); the bytes in use never exceed
 * the pool.  Batches run on their own streams (default priority), so requests overlap on the
 * device and a request that arrives while others run starts as soon as a stream and memory
 * free up.  Each trajectory's result depends only on (circuit, noise, its trajectory index
 * traj_base + t, dtype, plan): it is bit for bit the qs_run_trajectories result, alone or in
 * any mix.  All functions are thread-safe.  Times are seconds since qs_srv_create on a
 * monotonic clock.
 * ---------------------------------------------------------------------------------------- */
typedef struct qs_srv_s *qs_srv;

typedef struct {
    int32_t dtype;          /* qs_dtype of every request */
    int32_t max_inflight;   /* batches on the device at once (one stream each), 1..16 */
    int32_t max_chunk_traj; /* largest trajectory batch, <= 4096; <= 0 means 256 */
    int32_t reserved;
    qs_plan plan;           /* plan of every request, as in qs_run_trajectories */
} qs_srv_config;

typedef struct {
    int32_t status;         /* QS_OK, or the error that ended the request */
    int32_t n_chunks;       /* batches launched */
    int32_t chunk_traj;     /* trajectories per batch (the last may be fewer) */
    int32_t reserved;
    uint64_t chunk_bytes;   /* pool bytes one batch holds */
    double t_submit, t_admit, t_done;
    double latency_s;       /* t_done - t_submit */
    double queue_s;         /* t_admit - t_submit: wait for a stream and memory */
} qs_srv_job_info;

typedef struct {
    uint64_t submitted, completed, failed;
    uint64_t trajectories;     /* trajectories finished */
    uint64_t chunks;           /* batches launched */
    uint64_t admission_waits;  /* times the queue head found no free range large enough */
    uint64_t pool_bytes, peak_bytes, in_use_bytes;
    int32_t peak_inflight, inflight, queued, reserved;
    double busy_s;             /* time with at least one batch on the device */
    double elapsed_s;
} qs_srv_stats;

/* Start a server over pool[0, pool_bytes) (device memory, 256-byte aligned) on the pool's
 * device.  Creates max_inflight streams, events and pinned result buffers. */
qs_status qs_srv_create(const qs_srv_config *cfg, void *pool, size_t pool_bytes, qs_srv *out);
/* Queue one request: arguments as in qs_run_trajectories (gates, noise and e_per_traj are
 * copied).  Returns QS_ENOMEM when one trajectory does not fit the pool.  *job_out gets the
 * request id. */
qs_status qs_srv_submit(qs_srv srv, const qs_gate *gates, int n_gates, int n_qubits,
                        uint64_t init_index, const qs_noise *nz, int n_traj, int64_t marked,
                        uint64_t *job_out);
/* *done = 1 once every batch of the request has finished (or it failed). */
qs_status qs_srv_poll(qs_srv srv, uint64_t job, int *done);
/* Block until the request has finished; timeout_s < 0 waits without limit, else QS_EBUSY on
 * timeout. */
qs_status qs_srv_wait(qs_srv srv, uint64_t job, double timeout_s);
/* Results of a finished request (host arrays of n_traj doubles, each nullable; p_out needs
 * marked >= 0), and its timing; releases the request id.  Returns the request's error if it
 * failed (info is filled either way). */
qs_status qs_srv_result(qs_srv srv, uint64_t job, double *fid_out, double *p_out, double *norm_out,
                        qs_srv_job_info *info);
qs_status qs_srv_stats_get(qs_srv srv, qs_srv_stats *out);
/* Finish every queued request, then release streams, events and pinned buffers. */
qs_status qs_srv_destroy(qs_srv srv);

#ifdef __cplusplus
}
#endif

#endif /* QSIM_H */
