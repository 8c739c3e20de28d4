// Internal declarations shared by the host runtime and the gfx950 kernels of libqsim.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <memory>
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
//
// Per slot, a prep kernel writes one record per op of the pass (complex numbers in the
// amplitude precision): a one-qubit op's 2x2 matrix, and for its folded controlled phases
// (conditioned on the other qubit, applied to the |1> input = "pre" or output = "post"):
//   reg[RB]  phase factor per register bit,
//   lo[32]   product over the thread-id bits 0..4 that are set, indexed by tid & 31,
//   hi[16]   product over the thread-id bits 5..8 that are set, indexed by tid >> 5,
//   outer[n] the phases conditioned on tile-number bits (multiplied per tile in the kernel).
// ---------------------------------------------------------------------------------------
constexpr int kMaxTileBits = 15;
constexpr int kMaxRegBits = 4;
constexpr int kPhaseTable = 4 + 32 + 16;   // reg + lo + hi entries of a phase block

struct RoundDesc {
    uint32_t reg_mask;            // tile-local bits held in registers during this round
    int32_t op_begin;
    int32_t op_end;
    int32_t block_rec;            // -1: the ops run one by one; else the round runs as one dense
                                  // 16 x 16 block on the matrix cores, whose operand table (per
                                  // slot, 1024 floats in lane order) starts at this record entry
    uint32_t roff[16];            // tile-local offset of register r (32-bit: scalar loads)
    uint32_t sroff[16];           // lds_swizzle(roff[r])
    uint16_t tlo[32];             // tile-local bits of thread-id bits 0..4, indexed by tid & 31
    uint16_t thi[16];             // tile-local bits of thread-id bits 5..8, indexed by tid >> 5
    int32_t seq;                  // straight-line round: in a pass of the simple untouched-target
                                  // kind, k > 0 one-qubit ops on register bits k-1, ..., 0 in that
                                  // order; in a pass of the plain kind, on bits 0, ..., k-1, or
                                  // (9) two runs on bits 0..3 around one diagonal pattern
    int32_t reserved_;
};

// LDS slot of tile-local index l: the low four bits are xor-ed with the higher nibbles of l, a
// bijection (the high bits are unchanged) that spreads the accesses of a register layout over
// the banks: a 64-bit access serves 16 lanes per cycle, whose slots differ in the low four bits
// whenever the layout's four lowest thread bits lie in different positions of their nibbles
// (every layout of a contiguous register run, for instance).  It is linear over XOR, so for
// disjoint thread and register bits lds_swizzle(t | r) = lds_swizzle(t) ^ lds_swizzle(r).
__host__ __device__ inline uint32_t lds_swizzle(uint32_t l)
{
    return l ^ ((l >> 4) & 15u) ^ ((l >> 8) & 15u) ^ ((l >> 12) & 15u);
}

struct PassDesc {
    int32_t K;
    int32_t RB;
    int32_t round_begin;
    int32_t round_end;
    uint64_t outer_mask;          // physical bits (< n) that are not in the tile
    uint64_t classical;           // outer bits that no non-diagonal gate has touched before this
                                  // pass: they still hold the initial basis index's values, so a
                                  // tile whose bits there differ from it holds only zeros
    int32_t q_pos[16];            // tile-local bit j -> physical bit
    int32_t op_begin, op_end;     // the pass's ops (records)
    int32_t rec_size;             // complex entries of the pass's records per slot
    int32_t job_begin, job_end;   // OuterJobs of the pass (per-tile outer phase products)
    int32_t stage_begin, stage_end;
    int32_t load_round;           // index in the rounds array of the load layout (thread id in
                                  // the low tile-local bits), stored just before round_begin
    uint32_t lclassical;          // tile-local bits whose qubits no non-diagonal gate has touched
                                  // before this pass: only the amplitudes that agree with the
                                  // basis index there can be nonzero, and only those are read
    int32_t zero_fill;            // first pass: store the tiles outside the support as zeros
                                  // (needed unless the last pass rewrites every amplitude)
    int32_t uni_kernel;           // run the kernel variant with uniform factors for blocks
                                  // without thread-conditioned phases (most blocks are such)
    uint64_t reg_off[16];         // load layout: physical index bits of register r
    int32_t store_round;          // index in the rounds array of the layout the tile is stored
                                  // in: the pass's last round when its layout keeps the low run
                                  // bits in the thread id, else the load layout
    int32_t blocks;               // some round of the pass runs as a dense block (matrix cores)
    uint64_t store_off[16];       // store layout: physical index bits of register r
    int32_t zin_ops;              // one-qubit ops of the pass acting on a target that still holds
                                  // its basis bit (zero-input updates): 0 none, 1 some, 2 all,
                                  // 3 all, each with a real matrix, no input phase and at most
                                  // a uniform output factor; 4 none, each with a real matrix and
                                  // no folded phase; 5 the pass has no one-qubit op
    int32_t mixed_ops;            // the pass has ops other than one-qubit gates
};

// A stage: consecutive rounds whose records, outer jobs and outer bits stay within the
// per-stage bounds below (record and job offsets of ops are relative to the pass; stage ranges
// are absolute except rec_*, which are relative to the pass's record block).  The fused kernel
// walks stages as plain ranges of rounds; the bounds keep the descriptor tables of one stage
// small.
struct StageDesc {
    int32_t round_begin, round_end;
    int32_t op_begin, op_end;
    int32_t rec_begin, rec_end;
    int32_t job_begin, job_end;   // absolute OuterJob indices
    int32_t obits_begin, obits_end;
};

constexpr int kStageOps = 48;     // op descriptors per stage
constexpr int kStageJobs = 64;    // outer jobs per stage
constexpr int kStageObits = 512;  // outer condition bits per stage

enum OpType : int32_t { OP_U1 = 0, OP_U2 = 1, OP_DIAG = 2 };
enum DiagKind : int32_t { DIAG_NEGATE = 0, DIAG_PHASE = 1 };
enum PrepKind : int32_t { PR_REG = 0, PR_THREAD = 1, PR_OUTER = 2, PR_BASIS = 3 };

// OPF_REAL: the one-qubit matrix the kernel applies is real in every slot (for a two-qubit op:
// its 4 x 4 matrix is real).  OPF_CHAIN: the gate
// is an inner member of a phase chain (its table rows hold a real matrix and an input phase,
// written by the chain kernel).  OPF_UPHASE: the op has no folded input block, and its input
// phase is the uniform record entry rec + 4.  OPF_PREW: the op's input phase does not depend
// on register bits (a per-thread or uniform factor only).
// OPF_PRE_UNI / OPF_POST_UNI: the folded input / output block has no phase conditioned on a
// thread-id bit, so its per-thread factor is the same for every thread of a block.
// OPF_POSTW: the folded output block has no phase conditioned on a register bit (one factor
// for all the registers of a thread).
enum OpFlags : int32_t {
    OPF_REAL = 1, OPF_CHAIN = 2, OPF_UPHASE = 4, OPF_PREW = 8, OPF_PRE_UNI = 16, OPF_POST_UNI = 32,
    OPF_POSTW = 64
};

struct OpDesc {
    int32_t type;
    int32_t p0, p1;               // register-bit positions of the target(s)
    int32_t flags;
    int32_t rec;                  // record offset (complex entries) within the slot's block
    int32_t pre_rec, post_rec;    // phase blocks (-1: none)
    int32_t pre_job;              // OuterJob index within the pass (-1: none)
    int32_t post_job;
    int32_t gate;                 // gate index (noise-table row, matrix)
    int32_t pref_begin, pref_end; // PrepRefs of this op
    int32_t diag_kind;
    uint32_t lmask, lvalue;       // DIAG: tile-local condition (l & lmask) == lvalue
    // U1: register-index bits whose tile-local qubits no non-diagonal gate has touched before
    // this op (they still hold the run's basis bits, so registers that disagree there are zero)
    uint32_t creg;
    uint64_t omask, ovalue;       // DIAG: tile condition (outer index & omask) == ovalue
};

// A controlled phase folded into a one-qubit op: the phase of gate `gate` (noise table) when
// the condition bit is 1.  kind PR_REG: register bit `bit`; PR_THREAD: thread-id bit `bit`;
// PR_OUTER: stored at record entry `slot_entry`, conditioned per tile by an OuterJob;
// PR_BASIS: a tile-local condition qubit (physical bit `bit`) that no non-diagonal gate has
// touched yet, so every amplitude that can be nonzero holds the run's basis bit there: the
// phase is one factor for the whole block when that bit is 1 and none when it is 0 (the
// amplitudes it would otherwise reach are zero).
struct PrepRef {
    int32_t kind;
    int32_t post;
    int32_t bit;
    int32_t gate;
    int32_t slot_entry;
    int32_t reserved;
};

// Per tile: w = product of the record entries rec_off .. rec_off + n - 1 whose physical bit
// obits[bits_off + k] is set in the tile number.
struct OuterJob {
    int32_t op;
    int32_t rec_off;
    int32_t bits_off;
    int32_t n;
};

// ---------------------------------------------------------------------------------------
// Launchers (kernels.hip / fused.hip / fr.hip).  All asynchronous on `st`.
// Noise table: tab[(g * S + s) * 8 + 0..7] = complex 2x2 (U1) or phase in [0..1] (CP), FP64.
// ---------------------------------------------------------------------------------------
// Per-run values read from device memory by a replayed launch sequence (a captured graph
// keeps kernel arguments fixed): when a kernel gets a non-null RunParams pointer, these
// replace the seed, request, trajectory base, initial basis index and marked index.
struct RunParams {
    uint64_t seed;
    uint32_t request;
    uint32_t traj_base;
    int64_t init;                 // initial basis index (physical)
    int64_t marked;               // physical marked index, -1: none
};

struct NoiseArgs {
    const RunParams *dyn;         // nullptr: the fields below
    double e;                     // used when e_dev == nullptr
    const double *e_dev;          // per-slot strength (device, S entries) or nullptr
    uint64_t seed;
    uint32_t request;
    uint32_t traj_base;           // counter of slot first_noisy_slot
    int32_t first_noisy_slot;     // slots below this one are ideal (e = 0)
};

hipError_t launch_noise_table(const qs_gate *gates_dev, int n_gates, int S, NoiseArgs na,
                              double *tab, hipStream_t st);
// Rewrites the noise-table rows of the phase chains (chain layout in the fused path's
// documentation); chain_gates / chain_off in device memory, n_chains >= 1.
hipError_t launch_phase_chains(double *tab, int S, const int32_t *chain_gates, const int32_t *chain_off,
                               int n_chains, hipStream_t st);
hipError_t launch_noise_draw(uint64_t seed, uint32_t request, uint32_t stream,
                             const uint32_t *sites, int n_sites, uint32_t traj_base, int n_traj,
                             double *out, hipStream_t st);
hipError_t launch_init_basis(void *psi, qs_dtype dt, int n, int S, uint64_t index, hipStream_t st,
                             const RunParams *dyn = nullptr);
hipError_t launch_sweep_u1(void *psi, qs_dtype dt, int n, int S, int q, const double *tab_row,
                           hipStream_t st);
hipError_t launch_sweep_cp(void *psi, qs_dtype dt, int n, int S, int qa, int qb,
                           const double *tab_row, hipStream_t st);
hipError_t launch_sweep_perm(void *psi, qs_dtype dt, int n, int S, int kind, int qa, int qb,
                             hipStream_t st);
// m32: host 4x4 complex matrix (32 doubles), passed to the kernel by value.
// Dense 16x16 (m_dev: 256 complex FP64, device memory) on index bits bits[0..3] of one
// vector of nbits >= 4 qubits; local index bit k <-> index bit bits[k] (distinct).
hipError_t launch_sweep_4q(void *psi, qs_dtype dt, int nbits, const int bits[4], const double *m_dev,
                           hipStream_t st);
hipError_t launch_sweep_2q(void *psi, qs_dtype dt, int n, int S, int qa, int qb,
                           const double *m32, hipStream_t st);
// One gate's operator for S slots (as launch_noise_table for a single gate passed by value).
hipError_t launch_noise_one(const qs_gate &g, int S, NoiseArgs na, double *tab, hipStream_t st);
hipError_t launch_flip(void *psi, qs_dtype dt, int n, int S, uint64_t mask, uint64_t value,
                       hipStream_t st);
// Multiply the amplitudes with (index & mask) == value by fre + i fim.
hipError_t launch_scale_pattern(void *psi, qs_dtype dt, int n, int S, uint64_t mask, uint64_t value,
                                double fre, double fim, hipStream_t st);
// Per-slot (Re <ref|psi_s>, Im <ref|psi_s>, <psi_s|psi_s>, Re psi_s[marked], Im psi_s[marked])
// with ref = slot ref_slot of ref_psi; out has S * 5 doubles.  partials: reduce_partials_size.
size_t reduce_partials_doubles(int n, int S);
// Sums per-slot partials (2^log_blocks per slot, 3 doubles each) into out[slot * 5 ...] as
// launch_overlaps does (with the marked amplitude of psi).
hipError_t launch_overlap_final(const void *psi, qs_dtype dt, int n, int S, int log_blocks, int64_t marked,
                                const double *partials, double *out, hipStream_t st, const RunParams *dyn);
hipError_t launch_overlaps(const void *ref_psi, int ref_slot, const void *psi, qs_dtype dt, int n,
                           int S, int64_t marked, double *partials, double *out, hipStream_t st,
                           const RunParams *dyn = nullptr);
// <psi|rho|psi> and Tr rho over vec(rho) of n qubits: out = (Re f, Im f, Re tr, Im tr).
hipError_t launch_dm_expect(const void *rho, const void *psi, qs_dtype dt, int n,
                            double *partials, double *out, hipStream_t st);
hipError_t launch_copy(void *dst, const void *src, size_t bytes, hipStream_t st);
// dst[sigma(i)] = src[i] for the 2^n indices of one state, sigma moving index bit q to bit
// perm[q] (perm: host array of n distinct bits, n <= 40).
hipError_t launch_permute_bits(void *dst, const void *src, qs_dtype dt, int n, const int32_t *perm,
                               hipStream_t st);

struct ProgramDev {
    const PassDesc *passes;
    const StageDesc *stages;
    const RoundDesc *rounds;
    const OpDesc *ops;
    const PrepRef *prefs;
    const OuterJob *jobs;
    const int32_t *obits;
};

// Records of pass `pass_host` for all S slots into rec (S * rec_size complex entries).
hipError_t launch_pass_prep(qs_dtype dt, int S, const PassDesc *pass_host, ProgramDev prog,
                            const double *tab, const qs_gate *gates_dev, void *rec, int64_t basis,
                            const RunParams *dyn, hipStream_t st);
// Sets the fused kernels' LDS limit (done by the first launch otherwise); call before capturing
// a graph.
hipError_t fused_prepare_attributes();
// init >= 0: the first pass of a run, which makes |init> instead of reading the state; basis:
// the run's initial basis index (every pass, for the zero tiles of untouched qubits).
// wtab: the pass's per-tile products of the phases conditioned on tile-number bits, written by
// launch_pass_jobs (S * 2^(walked tile-number bits) * jobs entries).
// otab: the tile-number bits of each tile's physical index (2^(walked bits) entries), also
// written by launch_pass_jobs.
hipError_t launch_fused_pass(void *psi, qs_dtype dt, int n, int S, const PassDesc *pass_host,
                             int pass_index, int64_t init, int64_t basis, ProgramDev prog, const void *rec,
                             const void *wtab, const uint64_t *otab, hipStream_t st, const RunParams *dyn = nullptr,
                             double *ovl = nullptr, int slot_base = 0, int slots = 0);
// ovl (non-null): the pass runs only the slots [slot_base, slot_base + slots), tile-major, and
// also writes each (slot, tile) block's FP64 sums Re/Im <psi_0|psi_slot> and <psi_slot|psi_slot>
// to ovl[((slot << walked bits) | tile) * 3 ...]; slot 0's tiles must be final before a launch
// with slot_base > 0 (run slot 0 alone first).  Finished by launch_overlap_final.
// Walked tile-number bits of a pass launch (the tiles its blocks cover).
int fused_walked_bits(int n, const PassDesc *pass_host, int64_t init);
// The operand tables of the pass's block rounds (after launch_pass_prep of the pass; complex<float>
// plans only).
hipError_t launch_block_prep(qs_dtype dt, int S, const PassDesc *pass_host, ProgramDev prog, void *rec,
                             hipStream_t st);
// The per-tile products of a pass's outer jobs into wtab and the tiles' outer index bits into
// otab (after launch_pass_prep of the pass); the same init / basis / dyn as the pass's
// launch_fused_pass.
hipError_t launch_pass_jobs(qs_dtype dt, int n, int S, const PassDesc *pass_host, ProgramDev prog, const void *rec,
                            int64_t init, int64_t basis, const RunParams *dyn, void *wtab, uint64_t *otab,
                            hipStream_t st);
size_t fused_lds_bytes(qs_dtype dt, int K);
// Record entries per stage that fit next to a tile of 2^K amplitudes (two tiles per CU).
int stage_rec_cap(qs_dtype dt, int K);

// Fixed rank: Gram of the 2r half-columns; partial blocks then a fixed-order final sum.
size_t fr_gram_partials_doubles(int n, int r);
hipError_t launch_fr_gram(const void *V, qs_dtype dt, int n, int r, int q, double *partials,
                          double *gram_out, hipStream_t st);
hipError_t launch_fr_recombine(void *V, qs_dtype dt, int n, int r_in, int r_out, int q,
                               const double *coef_dev, hipStream_t st);
// Two-qubit Kraus sets: Gram of the 4r quarter-columns on (q0, q1) (32 x 32 complex, entry
// (x * 8 + c, y * 8 + d) with x = bit q0 + 2 bit q1) and the recombination with a 32 x 32
// coefficient matrix.
hipError_t launch_fr_gram2(const void *V, qs_dtype dt, int n, int r, int q0, int q1, double *partials,
                           double *gram_out, hipStream_t st);
hipError_t launch_fr_recombine2(void *V, qs_dtype dt, int n, int r_in, int r_out, int q0, int q1,
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
    std::vector<StageDesc> stages;
    std::vector<RoundDesc> rounds;
    std::vector<OpDesc> ops;
    std::vector<PrepRef> prefs;
    std::vector<OuterJob> jobs;
    std::vector<int32_t> obits;
    std::vector<int32_t> layout;  // logical qubit -> physical bit after the circuit
    // Phase chains: chain c is gates chain_gates[chain_off[c] .. chain_off[c + 1]), in circuit
    // order (empty: no chains; otherwise chain_off has one entry per chain plus one).
    std::vector<int32_t> chain_gates, chain_off;
    int K = 0, RB = 0;
    int max_rec = 0;              // largest per-slot record block of a pass (complex entries)
    int max_jobs = 0;             // most outer jobs of one pass
};

// mfma: run eligible register rounds as dense blocks on the matrix cores (RB = 4 only); phase
// chains are then not formed.
qs_status plan_fused(const qs_gate *gates, int n_gates, int n, int K, int RB, int run_bits,
                     int rec_cap, Program &out, bool mfma = false);

// Complex entries of one block round's operand table per slot (1024 floats).
constexpr int kBlockRecEntries = 512;

// A circuit validated and planned once; every batch of its trajectories reuses it.  The host
// arrays stay alive while any batch that copies from them is in flight.
struct TrajPrep {
    int n = 0;
    qs_dtype dt = QS_C64;
    bool fused = false;
    int K = 0, RB = 0;
    Program prog;
    std::vector<qs_gate> hg;       // device image of the gates (CNOT carries its 4x4 matrix)
    std::vector<int32_t> layout;   // logical qubit -> physical bit after the SWAP relabelling
    // host image of the fused program's tables (passes through chains) as they lie in the run
    // buffer: their offsets from the first table depend only on the table sizes, so one copy
    // uploads them all
    std::vector<char> prog_image;
};
// Validate and plan a trajectory run (cached per circuit, dtype and plan request);
// traj_prepare_uncached always plans.
qs_status traj_prepare_uncached(const qs_gate *gates, int n_gates, int n, qs_dtype dt, const qs_plan *plan,
                                TrajPrep &prep);

// One enqueued batch: `host` receives S*5 doubles (per slot: Re and Im of the overlap with the
// ideal slot, squared norm, Re and Im of the marked amplitude) when the stream reaches the copy.
struct TrajRun {
    int T = 0;
    std::vector<double> he;
    double *host = nullptr;
    std::vector<double> host_own;
};

qs_status traj_prepare(const qs_gate *gates, int n_gates, int n, qs_dtype dt, const qs_plan *plan,
                       TrajPrep &prep);
// The same without a copy: the cached preparation itself (kept alive by the pointer).
qs_status traj_prepare_shared(const qs_gate *gates, int n_gates, int n, qs_dtype dt, const qs_plan *plan,
                              std::shared_ptr<const TrajPrep> &prep);
size_t traj_prep_bytes(const TrajPrep &prep, int T);
qs_status traj_launch(const TrajPrep &prep, uint64_t init_index, const qs_noise *nz, int T, int64_t marked,
                      void *dev_buf, size_t buf_bytes, hipStream_t st, double *host_out, TrajRun &run);
void traj_finalize(const TrajPrep &prep, const TrajRun &run, double *fid_out, double *p_out, double *norm_out,
                   int32_t *layout_out);

inline size_t amp_bytes(qs_dtype dt) { return dt == QS_C64 ? 8 : 16; }
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
inline bool aligned256(const void *p) { return ((uintptr_t)p & 255u) == 0; }

}  // namespace qs
