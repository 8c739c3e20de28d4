// Fusion planner: turns a gate list into fused passes (see fused.hip).
//
// 1. SWAP gates become a relabelling of logical to physical qubits; no data moves.
// 2. Gates are grouped in order into passes; a pass may target at most `max_targets`
//    physical qubits with non-diagonal gates (one-qubit dense, two-qubit dense, CNOT).
//    Diagonal gates (controlled phases, sign flips) never close a pass.
// 3. A controlled phase on (c, t) commutes with everything between the previous and the next
//    non-diagonal gate on c or t.  It is folded into the next one-qubit gate on c or t as a
//    phase on that gate's |1> input (conditioned on the other qubit), else into the previous
//    one as a phase on its |1> output, else kept as a standalone diagonal op.
// 4. Each pass's tile is its targets plus the lowest remaining physical bits (for coalesced
//    rows of 2^run_bits amplitudes); its ops are grouped into register rounds of RB bits.
#include <algorithm>
#include <map>

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
};

int find_pos(const std::vector<int> &v, int x)
{
    for (size_t i = 0; i < v.size(); ++i)
        if (v[i] == x) return (int)i;
    return -1;
}

}  // namespace

qs_status plan_fused(const qs_gate *gates, int n_gates, int n, int K, int RB, int run_bits,
                     Program &P)
{
    if (K > n) K = n;
    if (K > kMaxTileBits) K = kMaxTileBits;
    if (RB > K) RB = K;
    if (RB > kMaxRegBits) RB = kMaxRegBits;
    if (K < 1 || RB < 1) return fail(QS_EINVAL, "fused plan: tile and register bits must be >= 1");
    if (K - RB > 9) return fail(QS_EINVAL, "fused plan: at most 512 threads per tile (tile_bits - reg_bits <= 9)");
    const bool whole = (n == K);
    int max_targets = whole ? K : K - run_bits;
    if (max_targets < 2) return fail(QS_EINVAL, "fused plan: tile too small for the run length");

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
        x.a = (G.kind == QS_G_FLIP) ? 0 : perm[G.q0];
        x.b = (G.kind == QS_G_CP || G.kind == QS_G_U2 || G.kind == QS_G_CNOT) ? perm[G.q1] : -1;
        x.gate = g;
        x.mask = x.value = 0;
        if (G.kind == QS_G_FLIP) {
            x.mask = map_mask(G.mask);
            x.value = map_mask(G.value);
        }
        pg.push_back(x);
    }
    P.layout = perm;

    // 2. passes
    std::vector<PassBuild> passes(1);
    std::vector<int> pass_of(pg.size(), 0);
    for (size_t i = 0; i < pg.size(); ++i) {
        const PG &x = pg[i];
        std::vector<int> need;
        if (x.kind == QS_G_U1) need = {x.a};
        else if (x.kind == QS_G_U2 || x.kind == QS_G_CNOT) need = {x.a, x.b};
        PassBuild *cur = &passes.back();
        int extra = 0;
        for (int q : need)
            if (find_pos(cur->targets, q) < 0) ++extra;
        if ((int)cur->targets.size() + extra > max_targets) {
            passes.emplace_back();
            cur = &passes.back();
        }
        for (int q : need)
            if (find_pos(cur->targets, q) < 0) cur->targets.push_back(q);
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
    std::vector<std::vector<Attach>> pre(pg.size()), post(pg.size());
    std::vector<bool> standalone(pg.size(), false);
    for (size_t i = 0; i < pg.size(); ++i) {
        const PG &x = pg[i];
        if (x.kind != QS_G_CP) {
            if (x.kind == QS_G_FLIP) standalone[i] = true;
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
        if (nx >= 0 && pg[nx].kind == QS_G_U1) {
            int cond = (pg[nx].a == x.a) ? x.b : x.a;
            pre[nx].push_back({cond, x.gate});
            continue;
        }
        int pa = prev_of(x.a), pb = prev_of(x.b);
        int px = std::max(pa, pb);
        if (px >= 0 && pg[px].kind == QS_G_U1) {
            int cond = (pg[px].a == x.a) ? x.b : x.a;
            post[px].push_back({cond, x.gate});
            continue;
        }
        standalone[i] = true;
    }

    // 4. tiles and rounds
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
        const uint32_t load_mask = ((1u << RB) - 1u) << (K - RB);

        // greedy register rounds
        struct RB_ { uint32_t need = 0; std::vector<int> ops; };
        std::vector<RB_> rounds(1);
        for (int i : ops_idx) {
            const PG &x = pg[i];
            uint32_t need = 0;
            if (x.kind == QS_G_U1) need = 1u << local_of[x.a];
            else if (x.kind == QS_G_U2 || x.kind == QS_G_CNOT) need = (1u << local_of[x.a]) | (1u << local_of[x.b]);
            uint32_t u = rounds.back().need | need;
            if (__builtin_popcount(u) > RB) {
                rounds.emplace_back();
                u = need;
            }
            rounds.back().need = u;
            rounds.back().ops.push_back(i);
        }
        pd.round_begin = (int)P.rounds.size();
        for (auto &rd : rounds) {
            // fill to RB bits: prefer the load-layout register bits, then the highest others
            uint32_t m = rd.need;
            for (int j = K - 1; j >= 0 && __builtin_popcount(m) < RB; --j)
                if ((load_mask >> j) & 1u) m |= 1u << j;
            for (int j = K - 1; j >= 0 && __builtin_popcount(m) < RB; --j) m |= 1u << j;
            RoundDesc R{};
            R.reg_mask = m;
            R.op_begin = (int)P.ops.size();
            int reg_index[32];
            {
                int k = 0;
                for (int j = 0; j < 32; ++j) reg_index[j] = ((m >> j) & 1u) ? k++ : -1;
            }
            auto classify = [&](int cond, int gate_idx) {
                PhaseRef pr{};
                pr.gate = gate_idx;
                int j = local_of[cond];
                if (j < 0) {
                    pr.cls = PH_OUTER;
                    pr.bit = cond;
                } else if (reg_index[j] >= 0) {
                    pr.cls = PH_REG;
                    pr.bit = reg_index[j];
                } else {
                    pr.cls = PH_THREAD;
                    pr.bit = j;
                }
                P.prefs.push_back(pr);
            };
            for (int i : rd.ops) {
                const PG &x = pg[i];
                OpDesc op{};
                op.gate = x.gate;
                if (x.kind == QS_G_U1) {
                    op.type = OP_U1;
                    op.p0 = reg_index[local_of[x.a]];
                    op.pre_begin = (int)P.prefs.size();
                    for (auto &at : pre[i]) classify(at.cond, at.gate);
                    op.pre_end = (int)P.prefs.size();
                    op.post_begin = (int)P.prefs.size();
                    for (auto &at : post[i]) classify(at.cond, at.gate);
                    op.post_end = (int)P.prefs.size();
                } else if (x.kind == QS_G_U2 || x.kind == QS_G_CNOT) {
                    op.type = OP_U2;
                    op.p0 = reg_index[local_of[x.a]];
                    op.p1 = reg_index[local_of[x.b]];
                } else {
                    op.type = OP_DIAG;
                    uint64_t mask, value;
                    if (x.kind == QS_G_FLIP) {
                        op.diag_kind = DIAG_NEGATE;
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
                }
                P.ops.push_back(op);
            }
            R.op_end = (int)P.ops.size();
            P.rounds.push_back(R);
        }
        pd.round_end = (int)P.rounds.size();
        P.passes.push_back(pd);
    }
    return QS_OK;
}

}  // namespace qs
