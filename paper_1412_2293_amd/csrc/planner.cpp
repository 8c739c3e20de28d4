// Fusion planner: turns a gate list into fused passes (see fused.hip).
//
// 1. SWAP gates become a relabelling of logical to physical qubits; no data moves.
// 2. Gates are grouped in order into passes; a pass may target at most `max_targets`
//    physical qubits above the low run bits with non-diagonal gates (one-qubit dense,
//    two-qubit dense, CNOT); targets among the run bits are free, as the tile always holds them.
//    Diagonal gates (controlled phases, sign flips) never close a pass.
// 3. A controlled phase on (c, t) commutes with everything between the previous and the next
//    non-diagonal gate on c or t.  It is folded into the next one-qubit gate on c or t as a
//    phase on that gate's |1> input (conditioned on the other qubit), else into the previous
//    one as a phase on its |1> output, else kept as a standalone diagonal op.
// 4. Each pass's tile is its targets plus the lowest remaining physical bits (for coalesced
//    rows of 2^run_bits amplitudes); its ops are grouped into register rounds of RB bits.
#include <algorithm>
#include <cmath>
#include <map>
#include <queue>

#include "internal.h"

namespace qs {

namespace {

struct PG {             // a gate on physical qubits
    int kind;
    int a, b;           // physical qubits
    int gate;           // index into the caller's gate list
    uint64_t mask, value;
    bool nondiag() const { return kind == QS_G_U1 || kind == QS_G_U2 || kind == QS_G_CNOT; }
};

struct Attach {         // controlled phase folded into a one-qubit gate
    int cond;           // physical condition qubit
    int gate;           // the controlled-phase gate index (its phase lives in the table)
};

struct PassBuild {
    std::vector<int> items;      // indices into the PG list, in order
    std::vector<int> targets;    // physical qubits touched non-diagonally
    int high = 0;                // targets outside the low run bits
};

// Qubits a gate acts on (a pattern gate: every qubit of its mask).
static void gate_qubits(const PG &x, int n, std::vector<int> &qs)
{
    qs.clear();
    if (x.kind == QS_G_FLIP || x.kind == QS_G_DIAG) {
        for (int q = 0; q < n; ++q)
            if ((x.mask >> q) & 1ull) qs.push_back(q);
        return;
    }
    qs.push_back(x.a);
    if (x.b >= 0) qs.push_back(x.b);
}

// List scheduling of the gates sel (indices into pg, in an order that respects the circuit)
// into groups.  Two gates commute when they act on disjoint qubits or are both diagonal, so
// the circuit fixes only a partial order: each gate follows the last non-diagonal gate on each
// of its qubits, and a non-diagonal gate also follows the diagonal gates on its qubits since
// then.  A group takes, lowest position in sel first, every gate whose predecessors are placed
// and whose targets still fit (at most cap targets for which counts(q) holds); a new group
// starts only when no such gate is left.  Appends the gates in the new order to order and the
// position where each group starts to starts.  The order of the gates on each qubit, and of a
// diagonal gate with respect to the non-diagonal gates on its qubits, is kept.
template <typename Counts>
static void list_schedule(const std::vector<PG> &pg, const std::vector<int> &sel, int n, int cap, Counts counts,
                          std::vector<int> &order, std::vector<int> &starts)
{
    const int m = (int)sel.size();
    std::vector<std::vector<int>> succ(m);
    std::vector<int> npred(m, 0), mark(m, -1), last_nd(n, -1);
    std::vector<std::vector<int>> diag_since(n);
    std::vector<int> qs;
    for (int i = 0; i < m; ++i) {
        const PG &x = pg[sel[i]];
        const bool nd = x.nondiag();
        gate_qubits(x, n, qs);
        auto dep = [&](int p) {
            if (p >= 0 && mark[p] != i) {
                mark[p] = i;
                succ[p].push_back(i);
                ++npred[i];
            }
        };
        for (int q : qs) {
            dep(last_nd[q]);
            if (nd)
                for (int d : diag_since[q]) dep(d);
        }
        for (int q : qs) {
            if (nd) {
                last_nd[q] = i;
                diag_since[q].clear();
            } else {
                diag_since[q].push_back(i);
            }
        }
    }
    std::priority_queue<int, std::vector<int>, std::greater<int>> ready;
    for (int i = 0; i < m; ++i)
        if (npred[i] == 0) ready.push(i);
    std::vector<char> in_group(n, 0);
    std::vector<int> group_targets, skipped;
    int placed = 0;
    while (placed < m) {
        starts.push_back((int)order.size());
        for (int q : group_targets) in_group[q] = 0;
        group_targets.clear();
        int used = 0;
        bool progress = true;
        while (progress) {
            // targets only grow within a group, so a gate passed over may fit once others have
            // added its qubits: scan again until nothing more is placed
            progress = false;
            skipped.clear();
            while (!ready.empty()) {
                const int i = ready.top();
                ready.pop();
                const PG &x = pg[sel[i]];
                int need[2], nn = 0;
                if (x.kind == QS_G_U1) need[nn++] = x.a;
                else if (x.kind == QS_G_U2 || x.kind == QS_G_CNOT) {
                    need[nn++] = x.a;
                    need[nn++] = x.b;
                }
                int extra = 0;
                for (int k = 0; k < nn; ++k)
                    if (!in_group[need[k]] && counts(need[k])) ++extra;
                if (used + extra > cap) {
                    skipped.push_back(i);
                    continue;
                }
                for (int k = 0; k < nn; ++k)
                    if (!in_group[need[k]]) {
                        in_group[need[k]] = 1;
                        group_targets.push_back(need[k]);
                        if (counts(need[k])) ++used;
                    }
                order.push_back(sel[i]);
                ++placed;
                progress = true;
                for (int sc : succ[i])
                    if (--npred[sc] == 0) ready.push(sc);
            }
            for (int i : skipped) ready.push(i);
        }
    }
}

// Gate order for the passes and their register rounds, by list scheduling over the circuit's
// partial order: first into passes (at most max_targets targets outside the low run bits,
// which every tile holds), then each pass's gates into rounds of at most RB target qubits.
// Taken strictly in circuit order a pass or a round ends at the first gate that does not fit,
// which costs a Grover iteration twice the passes, a layer of a random circuit on 30 qubits
// about three times the passes, and random layers twice the register rounds (each one more
// exchange through LDS).  The planner below cuts passes and rounds greedily in the new order,
// which reproduces these groups; the program computes the same state.  Plans with block rounds
// keep each pass in pass order: a block round needs every op's phases conditioned outside the
// registers to sit before the first or after the last op on its target, which rounds that span
// several layers of the same qubits rarely meet.
static void schedule_for_passes(std::vector<PG> &pg, int n, int max_targets, int run_bits, bool whole, int RB,
                                bool rounds)
{
    const int m = (int)pg.size();
    std::vector<int> all(m), by_pass, pass_starts;
    for (int i = 0; i < m; ++i) all[i] = i;
    list_schedule(pg, all, n, max_targets, [&](int q) { return whole || q >= run_bits; }, by_pass, pass_starts);
    pass_starts.push_back(m);
    std::vector<int> order, round_starts, seg;
    order.reserve(m);
    if (!rounds) order = by_pass;
    else
        for (size_t p = 0; p + 1 < pass_starts.size(); ++p) {
            seg.assign(by_pass.begin() + pass_starts[p], by_pass.begin() + pass_starts[p + 1]);
            list_schedule(pg, seg, n, RB, [](int) { return true; }, order, round_starts);
        }
    std::vector<PG> out;
    out.reserve(m);
    for (int i : order) out.push_back(pg[i]);
    pg.swap(out);
}

// Register offsets (plain and swizzled) and thread-id deposit tables of a round whose
// registers hold tile-local bits m.
RoundDesc make_round(uint32_t m, int K)
{
    RoundDesc R{};
    R.reg_mask = m;
    R.block_rec = -1;
    std::vector<int> regpos, tpos;
    for (int j = 0; j < K; ++j) ((m >> j) & 1u ? regpos : tpos).push_back(j);
    for (int r = 0; r < 16; ++r) {
        uint32_t o = 0;
        for (int k = 0; k < (int)regpos.size(); ++k)
            if ((r >> k) & 1) o |= 1u << regpos[k];
        R.roff[r] = o;
        R.sroff[r] = lds_swizzle(o);
    }
    for (int x = 0; x < 32; ++x) {
        uint32_t o = 0;
        for (int b = 0; b < 5 && b < (int)tpos.size(); ++b)
            if ((x >> b) & 1) o |= 1u << tpos[b];
        R.tlo[x] = (uint16_t)o;
    }
    for (int y = 0; y < 16; ++y) {
        uint32_t o = 0;
        for (int b = 0; b < 4 && 5 + b < (int)tpos.size(); ++b)
            if ((y >> b) & 1) o |= 1u << tpos[5 + b];
        R.thi[y] = (uint16_t)o;
    }
    return R;
}

int find_pos(const std::vector<int> &v, int x)
{
    for (size_t i = 0; i < v.size(); ++i)
        if (v[i] == x) return (int)i;
    return -1;
}

}  // namespace

qs_status plan_fused(const qs_gate *gates, int n_gates, int n, int K, int RB, int run_bits,
                     int rec_cap, Program &P, bool mfma)
{
    if (K > n) K = n;
    if (K > kMaxTileBits) K = kMaxTileBits;
    if (RB > K) RB = K;
    if (RB > kMaxRegBits) RB = kMaxRegBits;
    if (K < 1 || RB < 1) return fail(QS_EINVAL, "fused plan: tile and register bits must be >= 1");
    if (K - RB > 9) return fail(QS_EINVAL, "fused plan: at most 512 threads per tile (tile_bits - reg_bits <= 9)");
    if (RB == 4 && K - RB > 8)
        return fail(QS_EINVAL, "fused plan: reg_bits 4 allows at most 256 threads per tile (tile_bits <= 12)");
    const bool whole = (n == K);
    int max_targets = whole ? K : K - run_bits;
    bool two_qubit = false;
    for (int g = 0; g < n_gates; ++g)
        if (gates[g].kind == QS_G_U2 || gates[g].kind == QS_G_CNOT) two_qubit = true;
    if (max_targets < (two_qubit ? 2 : 1)) return fail(QS_EINVAL, "fused plan: tile too small for the run length");

    if (RB < 2)
        for (int g = 0; g < n_gates; ++g)
            if (gates[g].kind == QS_G_U2 || gates[g].kind == QS_G_CNOT)
                return fail(QS_EINVAL, "fused plan: two-qubit dense gates need reg_bits >= 2");
    P = Program();
    P.K = K;
    P.RB = RB;
    std::vector<int> perm(n);
    for (int q = 0; q < n; ++q) perm[q] = q;
    auto map_mask = [&](uint64_t m) {
        uint64_t o = 0;
        for (int q = 0; q < n; ++q)
            if (m & (1ull << q)) o |= 1ull << perm[q];
        return o;
    };

    // 1. physical gate list with SWAP relabelling
    std::vector<PG> pg;
    pg.reserve(n_gates);
    for (int g = 0; g < n_gates; ++g) {
        const qs_gate &G = gates[g];
        if (G.kind == QS_G_SWAP) {
            std::swap(perm[G.q0], perm[G.q1]);
            continue;
        }
        PG x;
        x.kind = G.kind;
        const bool pattern = G.kind == QS_G_FLIP || G.kind == QS_G_DIAG;
        x.a = pattern ? 0 : perm[G.q0];
        x.b = (G.kind == QS_G_CP || G.kind == QS_G_U2 || G.kind == QS_G_CNOT) ? perm[G.q1] : -1;
        x.gate = g;
        x.mask = x.value = 0;
        if (pattern) {
            x.mask = map_mask(G.mask);
            x.value = map_mask(G.value);
        }
        pg.push_back(x);
    }
    P.layout = perm;
    schedule_for_passes(pg, n, max_targets, run_bits, whole, RB, !mfma);

    // 1b. phase chains.  A unitary 2x2 matrix factors as M = e^{i phi} diag(1, e^{i beta}) R
    // diag(1, e^{i delta}) with R real.  The output factor diag(1, e^{i beta}) commutes with
    // every diagonal gate (controlled phases, sign flips) and with a CNOT on whose control it
    // sits, and a SWAP only relabels the wire (the physical bit stays), so it can be carried to
    // the next one-qubit gate on the same physical bit and multiplied into its matrix.  Along a
    // run of complex one-qubit gates on one wire every gate but the last then applies a real
    // matrix after a uniform input phase (half the multiplications of a complex one), and the
    // last absorbs the carried phase and the accumulated global phase.  A real gate, a CNOT
    // target or a dense two-qubit gate ends the run on its wire.
    std::vector<int8_t> chain_role(n_gates, 0);   // 1: inner member, 2: last member
    {
        auto chainable = [&](const qs_gate &G) {
            const double *m = G.m;
            bool real = true;
            for (int k = 1; k < 8; k += 2)
                if (m[k] != 0.0) real = false;
            if (real) return false;
            // unitary to within a few roundings: the factors reproduce M only then
            const double a[4][2] = {{m[0], m[1]}, {m[2], m[3]}, {m[4], m[5]}, {m[6], m[7]}};
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) {
                    // (M^dagger M)_{ij} = sum_k conj(M_ki) M_kj
                    double re = 0, im = 0;
                    for (int k = 0; k < 2; ++k) {
                        const double *x = a[2 * k + i], *y = a[2 * k + j];
                        re += x[0] * y[0] + x[1] * y[1];
                        im += x[0] * y[1] - x[1] * y[0];
                    }
                    if (std::fabs(re - (i == j ? 1.0 : 0.0)) > 1e-14 || std::fabs(im) > 1e-14) return false;
                }
            return true;
        };
        std::vector<std::vector<int32_t>> open(n);
        auto close = [&](int bit) {
            auto &c = open[bit];
            if (c.size() >= 2) {
                if (P.chain_off.empty()) P.chain_off.push_back(0);
                for (size_t k = 0; k < c.size(); ++k) chain_role[c[k]] = k + 1 < c.size() ? 1 : 2;
                P.chain_gates.insert(P.chain_gates.end(), c.begin(), c.end());
                P.chain_off.push_back((int32_t)P.chain_gates.size());
            }
            c.clear();
        };
        for (const PG &x : pg) {
            if (x.kind == QS_G_U1) {
                // block rounds take each gate's full complex matrix: no chains then
                if (!mfma && chainable(gates[x.gate])) open[x.a].push_back(x.gate);
                else close(x.a);
            } else if (x.kind == QS_G_CNOT) {
                close(x.b);
            } else if (x.kind == QS_G_U2) {
                close(x.a);
                close(x.b);
            }
        }
        for (int b = 0; b < n; ++b) close(b);
    }

    // 2. passes
    std::vector<PassBuild> passes(1);
    std::vector<int> pass_of(pg.size(), 0);
    for (size_t i = 0; i < pg.size(); ++i) {
        const PG &x = pg[i];
        std::vector<int> need;
        if (x.kind == QS_G_U1) need = {x.a};
        else if (x.kind == QS_G_U2 || x.kind == QS_G_CNOT) need = {x.a, x.b};
        PassBuild *cur = &passes.back();
        // the tile holds the targets and the low run bits: targets among the run bits are free
        int extra = 0;
        for (int q : need)
            if (find_pos(cur->targets, q) < 0 && (whole || q >= run_bits)) ++extra;
        if (cur->high + extra > max_targets) {
            passes.emplace_back();
            cur = &passes.back();
        }
        for (int q : need)
            if (find_pos(cur->targets, q) < 0) {
                cur->targets.push_back(q);
                if (whole || q >= run_bits) cur->high += 1;
            }
        cur->items.push_back((int)i);
        pass_of[i] = (int)passes.size() - 1;
    }

    // 3. fold controlled phases
    std::vector<std::vector<int>> nd_pos(n);   // positions of non-diagonal gates per qubit
    for (size_t i = 0; i < pg.size(); ++i) {
        const PG &x = pg[i];
        if (!x.nondiag()) continue;
        nd_pos[x.a].push_back((int)i);
        if (x.b >= 0) nd_pos[x.b].push_back((int)i);
    }
    std::vector<std::vector<Attach>> pre_att(pg.size()), post_att(pg.size());
    std::vector<bool> standalone(pg.size(), false);
    for (size_t i = 0; i < pg.size(); ++i) {
        const PG &x = pg[i];
        if (x.kind != QS_G_CP) {
            if (x.kind == QS_G_FLIP || x.kind == QS_G_DIAG) standalone[i] = true;
            continue;
        }
        auto next_of = [&](int q) {
            auto &v = nd_pos[q];
            auto it = std::upper_bound(v.begin(), v.end(), (int)i);
            return it == v.end() ? -1 : *it;
        };
        auto prev_of = [&](int q) {
            auto &v = nd_pos[q];
            auto it = std::lower_bound(v.begin(), v.end(), (int)i);
            return it == v.begin() ? -1 : *(it - 1);
        };
        int na = next_of(x.a), nb = next_of(x.b);
        int nx = (na < 0) ? nb : (nb < 0 ? na : std::min(na, nb));
        {
            // one qubit untouched so far (no non-diagonal gate before this one), the other's last
            // gate a one-qubit gate: fold as that gate's output phase conditioned on the untouched
            // qubit, which still holds the run's basis bit there, so the phase is one factor for
            // the whole tile (or none) instead of a per-amplitude input phase of the later gate
            const int pa = prev_of(x.a), pb = prev_of(x.b);
            const int pt = pa >= 0 && pb < 0 ? pa : (pb >= 0 && pa < 0 ? pb : -1);
            if (pt >= 0 && pg[pt].kind == QS_G_U1) {
                const int cond = (pg[pt].a == x.a) ? x.b : x.a;
                post_att[pt].push_back({cond, x.gate});
                continue;
            }
        }
        if (nx >= 0 && pg[nx].kind == QS_G_U1) {
            int cond = (pg[nx].a == x.a) ? x.b : x.a;
            pre_att[nx].push_back({cond, x.gate});
            continue;
        }
        int pa = prev_of(x.a), pb = prev_of(x.b);
        int px = std::max(pa, pb);
        if (px >= 0 && pg[px].kind == QS_G_U1) {
            int cond = (pg[px].a == x.a) ? x.b : x.a;
            post_att[px].push_back({cond, x.gate});
            continue;
        }
        standalone[i] = true;
    }

    // 4. tiles, rounds and per-slot records
    int max_rec = 0;
    uint64_t touched = 0;   // physical qubits targeted by non-diagonal gates of earlier passes
    for (size_t pi = 0; pi < passes.size(); ++pi) {
        PassBuild &pb = passes[pi];
        std::vector<int> ops_idx;
        for (int i : pb.items)
            if (pg[i].nondiag() || standalone[i]) ops_idx.push_back(i);
        if (ops_idx.empty()) continue;
        // tile qubits
        std::vector<int> Q = pb.targets;
        for (int q = 0; (int)Q.size() < K && q < n; ++q)
            if (find_pos(Q, q) < 0) Q.push_back(q);
        std::sort(Q.begin(), Q.end());
        PassDesc pd{};
        pd.K = K;
        pd.RB = RB;
        int local_of[64];
        for (int q = 0; q < 64; ++q) local_of[q] = -1;
        uint64_t qmask = 0;
        for (int j = 0; j < K; ++j) {
            pd.q_pos[j] = Q[j];
            local_of[Q[j]] = j;
            qmask |= 1ull << Q[j];
        }
        uint64_t nmask = (n >= 64) ? ~0ull : ((1ull << n) - 1);
        pd.outer_mask = nmask & ~qmask;
        pd.classical = pd.outer_mask & ~touched;
        pd.lclassical = 0;
        for (int j = 0; j < K; ++j)
            if (!((touched >> Q[j]) & 1ull)) pd.lclassical |= 1u << j;
        for (int q : pb.targets) touched |= 1ull << q;
        uint32_t lcls = pd.lclassical;   // tile-local bits untouched so far in this pass
        const uint32_t kmask = (1u << K) - 1u;
        // register layout the rounds are padded towards (the top tile-local bits)
        const uint32_t top_mask = ((1u << RB) - 1u) << (K - RB);
        const uint32_t load_mask = top_mask;

        // greedy register rounds, closed also when the current stage reaches its bounds
        auto fill = [&](uint32_t need) {
            uint32_t m = need;
            for (int j = K - 1; j >= 0 && __builtin_popcount(m) < RB; --j)
                if ((load_mask >> j) & 1u) m |= 1u << j;
            for (int j = K - 1; j >= 0 && __builtin_popcount(m) < RB; --j) m |= 1u << j;
            return m;
        };
        auto costs = [&](int i, int &rec_c, int &jobs_c, int &obits_c) {
            const PG &x = pg[i];
            rec_c = jobs_c = obits_c = 0;
            if (x.kind == QS_G_U1) {
                // the matrix, plus the uniform input phase of an inner chain member with no
                // folded input block
                rec_c = (chain_role[x.gate] == 1 && pre_att[i].empty()) ? 5 : 4;
                for (int post = 0; post < 2; ++post) {
                    const auto &att = (post ? post_att : pre_att)[i];
                    if (att.empty()) continue;
                    int no = 0;
                    for (auto &at : att)
                        if (local_of[at.cond] < 0) ++no;
                    rec_c += kPhaseTable + no;
                    if (no) {
                        ++jobs_c;
                        obits_c += no;
                    }
                }
            } else if (x.kind == QS_G_U2 || x.kind == QS_G_CNOT) {
                rec_c = 16;
            } else {
                rec_c = 1;
            }
        };
        struct RB_ { uint32_t need = 0; uint32_t forced = 0; bool stage_start = false; std::vector<int> ops; };
        std::vector<RB_> rounds(1);
        rounds.back().stage_start = true;
        int st_ops = 0, st_rec = 0, st_jobs = 0, st_obits = 0;
        for (int i : ops_idx) {
            const PG &x = pg[i];
            uint32_t need = 0;
            if (x.kind == QS_G_U1) need = 1u << local_of[x.a];
            else if (x.kind == QS_G_U2 || x.kind == QS_G_CNOT) need = (1u << local_of[x.a]) | (1u << local_of[x.b]);
            int rc, jc, oc;
            costs(i, rc, jc, oc);
            RB_ &cur = rounds.back();
            uint32_t cur_mask = cur.forced ? cur.forced : fill(cur.need);
            bool fits_reg = cur.forced ? ((need & ~cur.forced) == 0) : (__builtin_popcount(cur.need | need) <= RB);
            bool fits_stage = st_ops + 1 <= kStageOps && st_rec + rc <= rec_cap &&
                              st_jobs + jc <= kStageJobs && st_obits + oc <= kStageObits;
            if (!cur.ops.empty() && (!fits_reg || !fits_stage)) {
                RB_ nr;
                if (!fits_stage) {
                    nr.stage_start = true;
                    st_ops = st_rec = st_jobs = st_obits = 0;
                    if (fits_reg && cur_mask != 0 && (need & ~cur_mask) == 0) {
                        nr.forced = cur_mask;   // same register layout: no exchange
                        nr.need = cur.need;
                    }
                }
                if (!cur.forced) cur.forced = cur_mask;
                rounds.push_back(nr);
            }
            RB_ &r2 = rounds.back();
            if (!r2.forced) r2.need |= need;
            r2.ops.push_back(i);
            st_ops += 1;
            st_rec += rc;
            st_jobs += jc;
            st_obits += oc;
        }
        for (auto &rd : rounds)
            if (!rd.forced) rd.forced = fill(rd.need);
        // The layout the tile is loaded and stored in: the first round's, or else the last
        // round's, when it keeps the low run bits in the thread id (so that consecutive lanes
        // still read and write contiguous rows of 2^run_bits amplitudes); that saves the exchange
        // into the first round or out of the last.  Otherwise the top tile-local bits.
        // The tile is stored from the last round's layout under the same condition, which saves
        // the exchange back.
        uint32_t io_mask = top_mask;
        const uint32_t run_mask = whole ? 0u : ((1u << std::min(run_bits, K)) - 1u);
        const bool last_ok = (rounds.back().forced & run_mask) == 0;
        if ((rounds.front().forced & run_mask) == 0) io_mask = rounds.front().forced;
        else if (last_ok) io_mask = rounds.back().forced;
        const uint32_t st_mask = last_ok ? rounds.back().forced : io_mask;
        const RoundDesc load_rd = make_round(io_mask, K);
        auto phys_offsets = [&](uint32_t mask, uint64_t (&off)[16]) {
            int regpos[16], nr = 0;
            for (int j = 0; j < K; ++j)
                if ((mask >> j) & 1u) regpos[nr++] = j;
            for (int r = 0; r < 16; ++r) {
                uint64_t o = 0;
                for (int k = 0; k < nr; ++k)
                    if (r < (1 << RB) && ((r >> k) & 1)) o |= 1ull << Q[regpos[k]];
                off[r] = o;
            }
        };
        phys_offsets(io_mask, pd.reg_off);
        phys_offsets(st_mask, pd.store_off);
        pd.stage_begin = (int)P.stages.size();
        pd.load_round = (int)P.rounds.size();
        P.rounds.push_back(load_rd);
        pd.round_begin = (int)P.rounds.size();
        pd.op_begin = (int)P.ops.size();
        pd.job_begin = (int)P.jobs.size();
        int rec = 0;
        for (auto &rd : rounds) {
            uint32_t m = rd.forced;
            if (rd.stage_start) {
                if (P.stages.size() > (size_t)pd.stage_begin) {
                    StageDesc &prev = P.stages.back();
                    prev.round_end = (int)P.rounds.size();
                    prev.op_end = (int)P.ops.size();
                    prev.rec_end = rec;
                    prev.job_end = (int)P.jobs.size();
                    prev.obits_end = (int)P.obits.size();
                }
                StageDesc sd{};
                sd.round_begin = (int)P.rounds.size();
                sd.op_begin = (int)P.ops.size();
                sd.rec_begin = rec;
                sd.job_begin = (int)P.jobs.size();
                sd.obits_begin = (int)P.obits.size();
                P.stages.push_back(sd);
            }
            RoundDesc R = make_round(m, K);
            R.op_begin = (int)P.ops.size();
            int reg_index[32], tid_index[32];
            {
                int k = 0, t = 0;
                for (int j = 0; j < 32; ++j) {
                    bool in = j < K && ((m >> j) & 1u);
                    reg_index[j] = in ? k++ : -1;
                    tid_index[j] = (j < K && !in) ? t++ : -1;
                }
            }
            (void)kmask;
            for (int i : rd.ops) {
                const PG &x = pg[i];
                OpDesc op{};
                op.gate = x.gate;
                op.rec = rec;
                op.pre_rec = op.post_rec = -1;
                op.pre_job = op.post_job = -1;
                op.pref_begin = (int)P.prefs.size();
                if (x.kind == QS_G_U1) {
                    op.type = OP_U1;
                    op.p0 = reg_index[local_of[x.a]];
                    for (int j = 0; j < K; ++j)
                        if (((lcls >> j) & 1u) && reg_index[j] >= 0) op.creg |= 1u << reg_index[j];
                    lcls &= ~(1u << local_of[x.a]);
                    {
                        // U V(e xi) is real whenever U is: V of eq. (1) is a real rotation
                        bool real = true;
                        for (int k = 1; k < 8; k += 2)
                            if (gates[x.gate].m[k] != 0.0) real = false;
                        if (real) op.flags |= OPF_REAL;
                    }
                    rec += 4;
                    if (chain_role[x.gate] == 1) {
                        // inner chain member: real matrix; its input phase joins the folded
                        // input block, or takes record entry rec + 4 when there is none
                        op.flags |= OPF_REAL | OPF_CHAIN;
                        if (pre_att[i].empty()) {
                            op.flags |= OPF_UPHASE | OPF_PREW;
                            rec += 1;
                        }
                    }
                    for (int post = 0; post < 2; ++post) {
                        const auto &lst = post ? post_att : pre_att;
                        const auto &att = lst[i];
                        if (att.empty()) continue;
                        int block = rec;
                        int n_outer = 0;
                        for (auto &at : att)
                            if (local_of[at.cond] < 0) ++n_outer;
                        rec += kPhaseTable + n_outer;
                        if (post) op.post_rec = block; else op.pre_rec = block;
                        int outer_k = 0;
                        int bits_off = (int)P.obits.size();
                        for (auto &at : att) {
                            PrepRef pr{};
                            pr.post = post;
                            pr.gate = at.gate;
                            int j = local_of[at.cond];
                            if (j < 0) {
                                pr.kind = PR_OUTER;
                                pr.bit = at.cond;
                                pr.slot_entry = block + kPhaseTable + outer_k++;
                                P.obits.push_back(at.cond);
                            } else if ((lcls >> j) & 1u) {
                                pr.kind = PR_BASIS;
                                pr.bit = at.cond;
                            } else if (reg_index[j] >= 0) {
                                pr.kind = PR_REG;
                                pr.bit = reg_index[j];
                            } else {
                                pr.kind = PR_THREAD;
                                pr.bit = tid_index[j];
                            }
                            P.prefs.push_back(pr);
                        }
                        {
                            // which factors stay conditioned per register or per thread (the
                            // others: outer bits per tile, basis bits once per block)
                            bool reg = false, thr = false;
                            for (auto &at : att) {
                                const int j = local_of[at.cond];
                                if (j < 0 || ((lcls >> j) & 1u)) continue;
                                if (reg_index[j] >= 0) reg = true;
                                else thr = true;
                            }
                            if (!reg) op.flags |= post ? OPF_POSTW : OPF_PREW;
                            if (!thr) op.flags |= post ? OPF_POST_UNI : OPF_PRE_UNI;
                        }
                        if (n_outer > 0) {
                            OuterJob jb{};
                            jb.op = (int)P.ops.size();
                            jb.rec_off = block + kPhaseTable;
                            jb.bits_off = bits_off;
                            jb.n = n_outer;
                            if (post) op.post_job = (int)P.jobs.size() - pd.job_begin;
                            else op.pre_job = (int)P.jobs.size() - pd.job_begin;
                            P.jobs.push_back(jb);
                        }
                    }
                } else if (x.kind == QS_G_U2 || x.kind == QS_G_CNOT) {
                    op.type = OP_U2;
                    op.p0 = reg_index[local_of[x.a]];
                    op.p1 = reg_index[local_of[x.b]];
                    {
                        // a CNOT is a permutation; a dense gate is real when every entry is
                        bool real = true;
                        if (x.kind == QS_G_U2)
                            for (int k = 1; k < 32; k += 2)
                                if (gates[x.gate].m[k] != 0.0) real = false;
                        if (real) op.flags |= OPF_REAL;
                    }
                    lcls &= ~((1u << local_of[x.a]) | (1u << local_of[x.b]));
                    rec += 16;
                } else {
                    op.type = OP_DIAG;
                    uint64_t mask, value;
                    if (x.kind == QS_G_FLIP) {
                        op.diag_kind = DIAG_NEGATE;
                        mask = x.mask;
                        value = x.value;
                    } else if (x.kind == QS_G_DIAG) {
                        op.diag_kind = DIAG_PHASE;   // the factor comes from the gate's table row
                        mask = x.mask;
                        value = x.value;
                    } else {
                        op.diag_kind = DIAG_PHASE;
                        mask = (1ull << x.a) | (1ull << x.b);
                        value = mask;
                    }
                    uint32_t lm = 0, lv = 0;
                    for (int j = 0; j < K; ++j) {
                        if ((mask >> Q[j]) & 1ull) lm |= 1u << j;
                        if ((value >> Q[j]) & 1ull) lv |= 1u << j;
                    }
                    op.lmask = lm;
                    op.lvalue = lv;
                    op.omask = mask & pd.outer_mask;
                    op.ovalue = value & pd.outer_mask;
                    rec += 1;
                }
                op.pref_end = (int)P.prefs.size();
                P.ops.push_back(op);
            }
            R.op_end = (int)P.ops.size();
            // A round of one-qubit ops (at least three) on the four register bits runs as one dense
            // 16 x 16 block on the matrix cores: the ops' matrices and their phases conditioned on
            // register bits multiply into the block, in order.  A phase conditioned on a bit
            // outside the registers is diagonal on the op's target and commutes with the other
            // targets' ops, so it is applied before the block (an input phase) when no earlier op
            // of the round acts on that target, and after it (an output phase) when no later one
            // does; otherwise the round runs op by op.
            if (mfma && RB == 4 && K - RB >= 6 && R.op_end - R.op_begin >= 3) {
                bool ok = true;
                for (int oi = R.op_begin; ok && oi < R.op_end; ++oi) {
                    const OpDesc &o = P.ops[oi];
                    if (o.type != OP_U1 || (o.flags & (OPF_CHAIN | OPF_UPHASE))) {
                        ok = false;
                        break;
                    }
                    bool ext_pre = false, ext_post = false;
                    for (int k = o.pref_begin; k < o.pref_end; ++k)
                        if (P.prefs[k].kind != PR_REG) (P.prefs[k].post ? ext_post : ext_pre) = true;
                    for (int oj = R.op_begin; oj < R.op_end; ++oj) {
                        if (oj == oi || P.ops[oj].p0 != o.p0) continue;
                        if ((ext_pre && oj < oi) || (ext_post && oj > oi)) ok = false;
                    }
                }
                if (ok) {
                    R.block_rec = rec;
                    rec += kBlockRecEntries;
                }
            }
            P.rounds.push_back(R);
        }
        {
            // the uniform-factor kernel variant when most of the pass's blocks can use it
            int blocks = 0, uni = 0;
            for (int oi = pd.op_begin; oi < (int)P.ops.size(); ++oi) {
                const OpDesc &o = P.ops[oi];
                if (o.pre_rec >= 0) {
                    ++blocks;
                    uni += (o.flags & OPF_PRE_UNI) != 0;
                }
                if (o.post_rec >= 0) {
                    ++blocks;
                    uni += (o.flags & OPF_POST_UNI) != 0;
                }
            }
            pd.uni_kernel = blocks > 0 && 2 * uni > blocks;
        }
        {
            StageDesc &last = P.stages.back();
            last.round_end = (int)P.rounds.size();
            last.op_end = (int)P.ops.size();
            last.rec_end = rec;
            last.job_end = (int)P.jobs.size();
            last.obits_end = (int)P.obits.size();
        }
        pd.stage_end = (int)P.stages.size();
        pd.round_end = (int)P.rounds.size();
        pd.store_round = st_mask == io_mask ? pd.load_round : pd.round_end - 1;
        // a pass runs its rounds either all as blocks or all op by op (the kernel variants)
        {
            bool all = pd.round_end > pd.round_begin;
            for (int ri = pd.round_begin; ri < pd.round_end; ++ri)
                if (P.rounds[ri].block_rec < 0) all = false;
            if (!all)
                for (int ri = pd.round_begin; ri < pd.round_end; ++ri) P.rounds[ri].block_rec = -1;
            pd.blocks = all ? 1 : 0;
        }
        // which one-qubit ops of the pass find their target untouched (zero-input updates):
        // 0 none, 1 some, 2 all
        {
            int u1 = 0, zin = 0;
            for (int oi = pd.op_begin; oi < (int)P.ops.size(); ++oi)
                if (P.ops[oi].type == OP_U1) {
                    ++u1;
                    zin += ((P.ops[oi].creg >> P.ops[oi].p0) & 1u) != 0;
                }
            pd.zin_ops = zin == 0 ? 0 : (zin == u1 ? 2 : 1);
            pd.mixed_ops = u1 < (int)P.ops.size() - pd.op_begin ? 1 : 0;
            // 3: as 2, with only real matrices, no input phases and uniform output factors
            if (pd.zin_ops == 2 && !pd.mixed_ops && !pd.blocks) {
                bool simple = true;
                for (int oi = pd.op_begin; oi < (int)P.ops.size() && simple; ++oi) {
                    const OpDesc &o = P.ops[oi];
                    const int need = OPF_POSTW | OPF_POST_UNI;
                    if (!(o.flags & OPF_REAL) || (o.flags & (OPF_CHAIN | OPF_UPHASE)) || o.pre_rec >= 0 ||
                        (o.post_rec >= 0 && (o.flags & need) != need))
                        simple = false;
                }
                if (simple) pd.zin_ops = 3;
            }
            // 4: as 0, with only real matrices and no folded phases
            if (pd.zin_ops == 0 && !pd.blocks && u1 > 0) {
                bool plain = true;
                for (int oi = pd.op_begin; oi < (int)P.ops.size() && plain; ++oi) {
                    const OpDesc &o = P.ops[oi];
                    if (o.type != OP_U1) continue;
                    if (!(o.flags & OPF_REAL) || (o.flags & (OPF_CHAIN | OPF_UPHASE)) || o.pre_rec >= 0 ||
                        o.post_rec >= 0)
                        plain = false;
                }
                if (plain) pd.zin_ops = 4;
            }
            // 5: no one-qubit op at all
            if (u1 == 0 && pd.mixed_ops && !pd.blocks) pd.zin_ops = 5;
            // rounds that run as one straight-line sequence: in a pass of kind 3, k ops on
            // register bits k-1, ..., 0 in turn; of kind 4, on bits 0, ..., k-1, or two runs on
            // bits 0..3 around one diagonal pattern (seq = 9)
            for (int ri = pd.round_begin; ri < pd.round_end; ++ri) {
                RoundDesc &rd = P.rounds[ri];
                rd.seq = 0;
                const int k = rd.op_end - rd.op_begin;
                auto u1_at = [&](int i, int p) {
                    const OpDesc &o = P.ops[rd.op_begin + i];
                    return o.type == OP_U1 && o.p0 == p;
                };
                if (pd.zin_ops == 3 && k >= 1 && k <= RB) {
                    bool ok = true;
                    for (int i = 0; i < k; ++i) ok = ok && u1_at(i, k - 1 - i);
                    if (ok) rd.seq = k;
                } else if (pd.zin_ops == 4 && RB == 4) {
                    bool ok = k >= 1 && k <= RB;
                    for (int i = 0; ok && i < k; ++i) ok = u1_at(i, i);
                    if (ok) {
                        rd.seq = k;
                    } else if (k == 9 && P.ops[rd.op_begin + 4].type == OP_DIAG) {
                        ok = true;
                        for (int i = 0; i < 4; ++i) ok = ok && u1_at(i, i) && u1_at(5 + i, i);
                        if (ok) rd.seq = 9;
                    }
                }
            }
        }
        pd.op_end = (int)P.ops.size();
        pd.job_end = (int)P.jobs.size();
        pd.rec_size = rec;
        max_rec = std::max(max_rec, rec);
        P.max_jobs = std::max(P.max_jobs, pd.job_end - pd.job_begin);
        P.passes.push_back(pd);
    }
    // The first pass stores the zero tiles unless the last pass rewrites every amplitude (no
    // tile-number bit of it is still classical); every other pass reads only amplitudes of the
    // support, which the pass before it wrote.
    if (!P.passes.empty()) P.passes.front().zero_fill = P.passes.back().classical != 0;
    P.max_rec = max_rec;
    return QS_OK;
}

}  // namespace qs
