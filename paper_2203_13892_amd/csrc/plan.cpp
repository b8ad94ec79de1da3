// Pass planner: groups each subcircuit's gates into HBM passes over
// one-wave register tiles and prepares the per-op data the kernels read.
//
// A tile holds 2^(nl + nr) amplitudes of one trajectory: lane L of the wave
// owns the amplitudes whose physical qubits 0..nl-1 spell L (so every load
// and store of the wave is one contiguous run), and its register index j
// spells the nr register qubits.  A gate can run inside a pass when every
// qubit it changes is a lane or register qubit; a diagonal gate changes no
// qubit and runs anywhere.  Consecutive diagonal gates become one phase run:
// the product of diagonal unitaries is a phase polynomial of degree two in
// the index bits, evaluated per lane in fixed-point turns.
//
// Logical qubits sit at physical bit positions that change along the
// circuit: a swap gate only exchanges two positions (no data moves), and
// at the end of a pass the planner may exchange lane and register positions
// (a swap op inside the tile) so that the qubits the next gates change sit
// in lanes.  Gates are taken out of order when they commute: a gate may run
// before an earlier one that it shares no qubit with.  A noise event acts
// right after its gate in the order the pass runs, which is the circuit's
// own order on the gate's qubits, so every trajectory is unchanged.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <new>

#include "tqs_internal.h"

namespace tqs {

static bool is_zero(const cd &v) { return v.real() == 0.0 && v.imag() == 0.0; }

enum GateClass { GC_DIAG, GC_DENSE1, GC_CTRL, GC_DENSE2 };

// Diagonal, block-diagonal in one qubit (a control: its value never changes),
// or dense.
static GateClass classify(const Gate &g, uint32_t *ctrl) {
    const int k = 1 << g.a;
    bool diag = true;
    for (int r = 0; r < k; r++)
        for (int c = 0; c < k; c++)
            if (r != c && !is_zero(g.m[r * k + c])) diag = false;
    if (diag) return GC_DIAG;
    if (g.a == 1) return GC_DENSE1;
    for (int j = 0; j < 2; j++) {
        bool blk = true;
        for (int r = 0; r < 4; r++)
            for (int c = 0; c < 4; c++)
                if (((r >> j) & 1) != ((c >> j) & 1) && !is_zero(g.m[r * 4 + c])) blk = false;
        if (blk) {
            *ctrl = (uint32_t)j;
            return GC_CTRL;
        }
    }
    return GC_DENSE2;
}

// Qubits a gate changes (must be lane or register qubits of its pass).
static uint32_t changed_mask(const Gate &g, GateClass gc, uint32_t ctrl) {
    switch (gc) {
        case GC_DIAG: return 0;
        case GC_DENSE1: return 1u << g.q[0];
        case GC_CTRL: return 1u << g.q[1 - ctrl];
        case GC_DENSE2: return (1u << g.q[0]) | (1u << g.q[1]);
    }
    return 0;
}

// Phase of a unit complex number as 64-bit fixed-point turns.
static uint64_t turns_fixed(const cd &z) {
    long double t = std::atan2((long double)z.imag(), (long double)z.real()) /
                    (2.0L * 3.141592653589793238462643383279502884L);  // (-1/2, 1/2]
    if (t < 0) t += 1.0L;                                             // [0, 1)
    long double s = std::ldexp(t, 62);
    uint64_t v = (uint64_t)llroundl(s);
    return v << 2;  // wraps modulo one turn
}

constexpr uint32_t kNoGate = 0xFFFFFFFFu;  // a lane exchange inserted by the planner

struct PendingGate {
    uint32_t g;      // circuit gate, or kNoGate
    GateClass gc;
    uint32_t ctrl;
    uint32_t pq[2];  // physical positions of the gate's qubits when it runs
};

// The two-qubit swap (exactly): it only relabels positions.
static bool is_swap(const Gate &g) {
    if (g.a != 2) return false;
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++) {
            const bool one = (r == c && (r == 0 || r == 3)) || (r == 1 && c == 2) || (r == 2 && c == 1);
            if (g.m[r * 4 + c] != cd(one ? 1.0 : 0.0, 0.0)) return false;
        }
    return true;
}

static const cd kSwapMat[16] = {1, 0, 0, 0, 0, 0, 1, 0, 0, 1, 0, 0, 0, 0, 0, 1};

// Estimated lane instructions per amplitude of each op (used to bound the
// work of one pass to about what its HBM traffic takes).
static double op_cost(GateClass gc, bool lane_target, bool lane_other) {
    switch (gc) {
        case GC_DENSE1: return lane_target ? 10 : 5;
        case GC_CTRL: return lane_target ? 11 : 7;
        case GC_DENSE2: return lane_target && lane_other ? 26 : (lane_target || lane_other ? 20 : 17);
        case GC_DIAG: return 0;
    }
    return 0;
}

}  // namespace tqs

using namespace tqs;

#define TQS_GUARD_BEGIN try {
#define TQS_GUARD_END                                         \
    }                                                         \
    catch (const std::bad_alloc &) {                          \
        return fail(TQS_E_OOM, "host allocation failed");     \
    }                                                         \
    catch (...) {                                             \
        return fail(TQS_E_ARG, "unexpected exception");       \
    }

// One plan for a fully resolved level_exchange choice (tqs_plan_create below
// picks it when the tuning leaves it open).
static tqs_status plan_create_one(const tqs_circuit *c, const tqs_tree *tree, tqs_precision prec,
                                  const tqs_tuning *tuning, tqs_plan **out) {
    TQS_GUARD_BEGIN
    if (!c || !out) return fail(TQS_E_ARG, "circuit or out is NULL");
    *out = nullptr;
    if (prec != TQS_C64 && prec != TQS_C128) return fail(TQS_E_ARG, "unknown precision %d", (int)prec);
    std::vector<uint64_t> A;
    std::vector<uint32_t> cut;
    tqs_status st = validate_tree(tree, (uint32_t)c->gates.size(), &A, &cut);
    if (st) return st;
    tqs_tuning tu{};
    if (tuning) tu = *tuning;
    if (!tu.tile_qubits) tu.tile_qubits = prec == TQS_C64 ? 11 : 10;
    if (!tu.max_ops_per_pass) tu.max_ops_per_pass = 1024;
    if (!tu.chunk_states) {
        // launches of up to 8 GiB of states (1024 of 20 qubits): fewer, larger
        // launches; beyond that a leaf chunk's parents no longer stay in the
        // caches while it runs (measured on the 20-qubit QFT tree (16, 32, 32):
        // 575K shots/s at 512, 605K at 1024, 617K at 2048 with the pass at
        // 0.69, 0.69 and 0.66 of the HBM peak)
        const uint64_t state_bytes = (uint64_t)(prec == TQS_C64 ? 8 : 16) << c->n;
        tu.chunk_states = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(1024, (8ull << 30) / state_bytes));
    }
    if (!tu.sample_block_log) tu.sample_block_log = 12;
    if (!tu.pass_cost) tu.pass_cost = 480;
    if (tu.jit > 2) return fail(TQS_E_ARG, "jit must be 0 (default), 1 (on) or 2 (off)");
    if (!tu.jit) tu.jit = c->n >= 16 ? 1u : 2u;
    if (!tu.mfma_min_ops) tu.mfma_min_ops = 6;
    if (tu.lds_levels > 2) return fail(TQS_E_ARG, "lds_levels must be 0 (default), 1 (on) or 2 (off)");
    if (!tu.lds_levels) tu.lds_levels = 2;
    if (tu.level_exchange > 2) return fail(TQS_E_ARG, "level_exchange must be 0 (default), 1 (on) or 2 (off)");
    if (!tu.level_exchange) tu.level_exchange = 2;
    const uint32_t tmax = prec == TQS_C64 ? 12 : 11;
    if (tu.tile_qubits < 10 || tu.tile_qubits > tmax)
        return fail(TQS_E_ARG, "tile_qubits must be in 10..%u at this precision", tmax);
    if (tu.sample_block_log < 8 || tu.sample_block_log > 16)
        return fail(TQS_E_ARG, "sample_block_log must be in 8..16");
    if (tu.max_ops_per_pass > 60000) return fail(TQS_E_ARG, "max_ops_per_pass must be <= 60000");

    tqs_plan *p = new tqs_plan;
    p->n = c->n;
    p->prec = prec;
    p->tune = tu;
    p->arity = A;
    p->cut = cut;
    p->n_gates = (uint32_t)c->gates.size();
    p->reg_bits = tu.tile_qubits - kLaneBits;
    const uint32_t L = (uint32_t)A.size();
    uint64_t off = 0;
    for (uint32_t l = 0; l < L; l++) {
        p->level_offset.push_back(off);
        p->level_nodes.push_back(level_nodes(A, l));
        off += p->level_nodes.back();
    }
    p->n_nodes = off;
    p->n_leaves = p->level_nodes.back();
    p->sample_b = std::min(c->n, tu.sample_block_log);
    p->gate_pass.assign(p->n_gates, 0);
    p->gate_pos.assign(p->n_gates, 0);
    p->gate_q0.assign(p->n_gates, 0);
    p->gate_q1.assign(p->n_gates, 0);
    p->gate_a.assign(p->n_gates, 0);

    const uint32_t n = c->n;
    const uint32_t nl = std::min(n, kLaneBits);
    const uint32_t nr_max = std::min(n - nl, p->reg_bits);
    const uint32_t lane_mask = (1u << nl) - 1u;

    // the planner's permutation of qubit positions: lay[logical] = physical
    std::vector<uint32_t> lay(n), inv(n);
    for (uint32_t q = 0; q < n; q++) lay[q] = inv[q] = q;
    auto swap_pos = [&](uint32_t pa, uint32_t pb) {
        const uint32_t qa = inv[pa], qb = inv[pb];
        lay[qa] = pb;
        lay[qb] = pa;
        inv[pa] = qb;
        inv[pb] = qa;
    };
    std::vector<GateClass> cls(p->n_gates);
    std::vector<uint32_t> ctl(p->n_gates, 0);
    std::vector<char> swp(p->n_gates, 0);
    for (uint32_t gi = 0; gi < p->n_gates; gi++) {
        cls[gi] = classify(c->gates[gi], &ctl[gi]);
        swp[gi] = is_swap(c->gates[gi]) ? 1 : 0;
    }

    std::vector<PendingGate> pend;
    uint32_t pend_regs = 0;     // physical register positions the pass needs
    double pend_cost = 4.0;     // load + store
    uint32_t pend_lds = 0;      // bytes of the pass's staged op data
    const uint32_t amp_bytes = prec == TQS_C64 ? 8 : 16;

    auto emit = [&]() {
        PassDesc d;
        std::memset(&d, 0, sizeof d);
        d.nl = (uint8_t)nl;
        // register qubits: the needed positions, then the lowest others
        uint32_t regs = pend_regs;
        for (uint32_t b = nl; b < n && (uint32_t)__builtin_popcount(regs) < nr_max; b++) regs |= 1u << b;
        uint8_t role[32], pos[32];
        for (uint32_t b = 0; b < n; b++) {
            role[b] = ROLE_FIXED;
            pos[b] = (uint8_t)b;
        }
        for (uint32_t b = 0; b < nl; b++) {
            role[b] = ROLE_LANE;
            pos[b] = (uint8_t)b;
        }
        d.nr = 0;
        for (uint32_t b = nl; b < n; b++)
            if ((regs >> b) & 1) {
                role[b] = ROLE_REG;
                pos[b] = d.nr;
                d.rq[d.nr++] = (uint8_t)b;
            }
        d.nfree = 0;
        for (uint32_t b = 0; b < n; b++)
            if (role[b] == ROLE_FIXED) d.fbits[d.nfree++] = (uint8_t)b;
        d.op_begin = (uint32_t)p->ops.size();
        d.mat_begin = (uint32_t)p->mats.size();
        d.term_begin = (uint32_t)p->terms.size();

        size_t i = 0;
        while (i < pend.size()) {
            OpDesc o;
            std::memset(&o, 0, sizeof o);
            o.slot0 = (uint16_t)i;
            if (pend[i].gc == GC_DIAG) {
                // maximal run of consecutive diagonal gates
                size_t j = i;
                while (j < pend.size() && pend[j].gc == GC_DIAG) j++;
                o.kind = OP_DIAGRUN;
                o.slot1 = (uint16_t)j;
                o.mat = (uint32_t)p->mats.size();
                o.terms = (uint32_t)p->terms.size();
                o.gates = (uint32_t)p->dgates.size();
                // register-only gates fold into a table over the register
                // index; the others become phase terms, normalised so that
                // qubit 0 is the fixed or lane one and, for a term with a
                // register qubit, r = y0 + 2 x_reg, then grouped by role
                const uint32_t nt = 1u << d.nr;
                std::vector<cd> tab(nt, cd(1.0, 0.0));
                bool has_t = false;
                std::vector<DiagTerm> g_fix, g_lane, g_fixreg[kMaxRegBits], g_lanereg[kMaxRegBits];
                auto phase_fixed = [&](const cd &z) {
                    const uint64_t t64 = turns_fixed(z);
                    // complex64 runs keep 32-bit turns (rounded), complex128 runs 64-bit
                    return prec == TQS_C64 ? (uint64_t)(uint32_t)((t64 + 0x80000000ull) >> 32) : t64;
                };
                for (size_t k = i; k < j; k++) {
                    const Gate &g = c->gates[pend[k].g];
                    const uint32_t *pq = pend[k].pq;
                    const uint32_t nd = 1u << g.a;
                    DiagGate dg;
                    std::memset(&dg, 0, sizeof dg);
                    dg.nq = (uint8_t)g.a;
                    uint32_t nreg = 0, nlane = 0;
                    for (uint32_t q = 0; q < g.a; q++) {
                        dg.role[q] = role[pq[q]];
                        dg.pos[q] = pos[pq[q]];
                        dg.phys[q] = (uint8_t)pq[q];
                        if (role[pq[q]] == ROLE_REG) nreg++;
                        if (role[pq[q]] == ROLE_LANE) nlane++;
                    }
                    p->dgates.push_back(dg);
                    if (nreg == g.a) {
                        for (uint32_t t = 0; t < nt; t++) {
                            uint32_t r = 0;
                            for (uint32_t q = 0; q < g.a; q++) r |= ((t >> pos[pq[q]]) & 1u) << q;
                            tab[t] *= g.m[r * nd + r];
                        }
                        has_t = true;
                        continue;
                    }
                    DiagTerm tm;
                    std::memset(&tm, 0, sizeof tm);
                    tm.nq = (uint8_t)g.a;
                    // order: qubit 0 = a lane qubit if any, else a fixed one
                    uint32_t q0 = 0;
                    if (g.a == 2) {
                        const uint32_t r0 = role[pq[0]], r1 = role[pq[1]];
                        if (r0 == ROLE_REG || (r0 == ROLE_FIXED && r1 == ROLE_LANE)) q0 = 1;
                    }
                    const uint32_t q1 = 1 - q0;
                    tm.role[0] = role[pq[q0]];
                    tm.pos[0] = pos[pq[q0]];
                    tm.phys[0] = (uint8_t)pq[q0];
                    if (g.a == 2) {
                        tm.role[1] = role[pq[q1]];
                        tm.pos[1] = pos[pq[q1]];
                        tm.phys[1] = (uint8_t)pq[q1];
                    }
                    for (uint32_t r = 0; r < nd; r++) {
                        // r in the normalised order -> index in the gate's order
                        uint32_t rg = r;
                        if (g.a == 2 && q0 == 1) rg = ((r & 1u) << 1) | (r >> 1);
                        tm.th[r] = phase_fixed(g.m[rg * nd + rg]);
                    }
                    // the gate's index in the run (events inside a run split it)
                    tm.k = (uint8_t)std::min<size_t>(k - i, 255);
                    const bool reg1 = g.a == 2 && tm.role[1] == ROLE_REG;
                    if (nlane == 0) {
                        if (reg1) g_fixreg[tm.pos[1]].push_back(tm);
                        else g_fix.push_back(tm);
                    } else {
                        if (reg1) g_lanereg[tm.pos[1]].push_back(tm);
                        else g_lane.push_back(tm);
                    }
                }
                o.has_t = has_t ? 1 : 0;
                o.lam_mask = 0;
                for (uint32_t b = 0; b < kMaxRegBits; b++)
                    if (!g_fixreg[b].empty() || !g_lanereg[b].empty()) o.lam_mask |= (uint8_t)(1u << b);
                o.n_fix = (uint16_t)g_fix.size();
                o.n_lane = (uint16_t)g_lane.size();
                for (const DiagTerm &tm : g_fix) p->terms.push_back(tm);
                for (uint32_t b = 0; b < kMaxRegBits; b++) {
                    o.n_fixreg[b] = (uint16_t)g_fixreg[b].size();
                    for (const DiagTerm &tm : g_fixreg[b]) p->terms.push_back(tm);
                }
                for (const DiagTerm &tm : g_lane) p->terms.push_back(tm);
                for (uint32_t b = 0; b < kMaxRegBits; b++) {
                    o.n_lanereg[b] = (uint16_t)g_lanereg[b].size();
                    for (const DiagTerm &tm : g_lanereg[b]) p->terms.push_back(tm);
                }
                o.tmask = 0;  // (entries from 32 on are always applied)
                for (uint32_t t = 0; t < std::min(nt, 32u); t++)
                    if (tab[t] != cd(1.0, 0.0)) o.tmask |= 1u << t;
                o.ngates = (uint32_t)(j - i);
                for (uint32_t t = 0; t < nt; t++) p->mats.push_back(tab[t]);
                // per-gate diagonal entries for the gate-by-gate path
                for (size_t k = i; k < j; k++) {
                    const Gate &g = c->gates[pend[k].g];
                    const uint32_t nd = 1u << g.a;
                    p->dgates[o.gates + (k - i)].d = (uint32_t)p->mats.size();
                    for (uint32_t r = 0; r < nd; r++) p->mats.push_back(g.m[r * nd + r]);
                }
                i = j;
            } else {
                const bool ins = pend[i].g == kNoGate;
                const uint32_t a = ins ? 2u : c->gates[pend[i].g].a;
                const cd *m = ins ? kSwapMat : c->gates[pend[i].g].m;
                o.slot1 = (uint16_t)(i + 1);
                o.nq = (uint8_t)a;
                for (uint32_t q = 0; q < a; q++) {
                    o.role[q] = role[pend[i].pq[q]];
                    o.pos[q] = pos[pend[i].pq[q]];
                    o.phys[q] = (uint8_t)pend[i].pq[q];
                }
                o.kind = pend[i].gc == GC_DENSE2 ? OP_DENSE2 : OP_DENSE1;
                o.tq = pend[i].gc == GC_CTRL ? (uint8_t)(1 - pend[i].ctrl) : 0;
                o.mat = (uint32_t)p->mats.size();
                const uint32_t nd = 1u << a;
                o.real = 1;
                for (uint32_t r = 0; r < nd * nd; r++) {
                    p->mats.push_back(m[r]);
                    if (m[r].imag() != 0.0) o.real = 0;
                }
                i++;
            }
            p->ops.push_back(o);
        }
        d.op_count = (uint32_t)p->ops.size() - d.op_begin;
        d.mat_count = (uint32_t)p->mats.size() - d.mat_begin;
        d.term_count = (uint32_t)p->terms.size() - d.term_begin;
        d.has_d2 = 0;
        for (uint32_t k = d.op_begin; k < (uint32_t)p->ops.size(); k++)
            if (p->ops[k].kind == OP_DENSE2) d.has_d2 = 1;
        p->passes.push_back(d);
        pend.clear();
        pend_regs = 0;
        pend_cost = 4.0;
        pend_lds = 0;
    };

    const double diag_setup = 14.0 + 0.7 * (nr_max + 1);
    const double lane_swap_cost = 12.0;
    for (uint32_t l = 0; l < L; l++) {
        tqs::Level lv;
        lv.pass_begin = (uint32_t)p->passes.size();
        lv.g0 = cut[l];
        lv.g1 = cut[l + 1];
        std::vector<uint32_t> rem;
        for (uint32_t gi = cut[l]; gi < cut[l + 1]; gi++) rem.push_back(gi);
        // every level has at least one pass: its first pass copies the parent
        bool first_pass = true;
        while (first_pass || !rem.empty()) {
            first_pass = false;
            bool in_diag_run = false;
            uint32_t blocked = 0;  // logical qubits of gates left for later passes
            std::vector<uint32_t> left;
            for (uint32_t gi : rem) {
                const Gate &g = c->gates[gi];
                const uint32_t qm = (1u << g.q[0]) | (g.a == 2 ? 1u << g.q[1] : 0u);
                if (qm & blocked) {
                    blocked |= qm;
                    left.push_back(gi);
                    continue;
                }
                p->gate_a[gi] = g.a;
                if (swp[gi]) {
                    // relabel: the two logical qubits exchange positions
                    swap_pos(lay[g.q[0]], lay[g.q[1]]);
                    p->gate_pass[gi] = (uint32_t)p->passes.size();
                    p->gate_pos[gi] = (uint32_t)pend.size();
                    p->gate_q0[gi] = lay[g.q[0]];
                    p->gate_q1[gi] = lay[g.q[1]];
                    continue;
                }
                const GateClass gc = cls[gi];
                const uint32_t ctrl = ctl[gi];
                uint32_t chl = changed_mask(g, gc, ctrl), ch = 0;
                for (uint32_t q = 0; q < n; q++)
                    if ((chl >> q) & 1u) ch |= 1u << lay[q];
                ch &= ~lane_mask;
                const uint32_t need = (uint32_t)__builtin_popcount(pend_regs | ch);
                double cost;
                if (gc == GC_DIAG) {
                    // a new run pays its per-amplitude evaluation; each term adds
                    // per-lane work spread over the lane's amplitudes
                    cost = (in_diag_run ? 0.0 : diag_setup) + 0.2;
                } else {
                    const uint32_t tq = gc == GC_CTRL ? 1 - ctrl : 0;
                    const bool lt = lay[g.q[tq]] < nl;
                    const bool lo = g.a == 2 && lay[g.q[1 - tq]] < nl;
                    cost = op_cost(gc, lt, lo);
                }
                // staged bytes: op record, matrix or diagonal, phase term, run table
                uint32_t lds = 0;
                if (gc == GC_DIAG)
                    lds = (uint32_t)(sizeof(DiagTerm) + 4 * amp_bytes) +
                          (in_diag_run ? 0u : (uint32_t)sizeof(OpDesc) + (amp_bytes << nr_max));
                else
                    lds = (uint32_t)sizeof(OpDesc) + (g.a == 2 ? 16u : 4u) * amp_bytes;
                if (!pend.empty() && (need > nr_max || pend_cost + cost > tu.pass_cost ||
                                      pend_lds + lds > kPassLdsBytes ||
                                      pend.size() >= tu.max_ops_per_pass || pend.size() >= 60000)) {
                    blocked |= qm;
                    left.push_back(gi);
                    continue;
                }
                in_diag_run = (gc == GC_DIAG);
                pend_regs |= ch;
                pend_cost += cost;
                pend_lds += lds;
                PendingGate pg{gi, gc, ctrl, {lay[g.q[0]], g.a == 2 ? lay[g.q[1]] : lay[g.q[0]]}};
                pend.push_back(pg);
                p->gate_pass[gi] = (uint32_t)p->passes.size();
                p->gate_pos[gi] = (uint32_t)pend.size();  // slot after this gate
                p->gate_q0[gi] = pg.pq[0];
                p->gate_q1[gi] = pg.pq[1];
            }
            rem.swap(left);
            // the gates the exchange below prepares for: the level's remaining
            // gates, or (tuning level_exchange), after its last pass, the next
            // level's when the qubits they change would not fit the lanes plus
            // the register slots of one tile.  Tail events of this level then
            // precede an op, so fewer of its nodes may share a state.
            std::vector<uint32_t> ahead;
            if (!rem.empty()) {
                ahead = rem;
            } else if (tu.level_exchange == 1 && l + 1 < L) {
                uint32_t chp = 0;
                for (uint32_t gi = cut[l + 1]; gi < cut[l + 2]; gi++) {
                    if (swp[gi]) continue;
                    const uint32_t chl = changed_mask(c->gates[gi], cls[gi], ctl[gi]);
                    for (uint32_t q = 0; q < n; q++)
                        if ((chl >> q) & 1u) chp |= 1u << lay[q];
                }
                if ((uint32_t)__builtin_popcount(chp & ~lane_mask) > nr_max)
                    for (uint32_t gi = cut[l + 1]; gi < cut[l + 2]; gi++) ahead.push_back(gi);
            }
            if (!ahead.empty() && nl == kLaneBits && n > nl) {
                // the logical qubits the next gates change, in order of need
                std::vector<uint32_t> need;
                uint32_t needm = 0;
                for (uint32_t gi : ahead) {
                    const Gate &g = c->gates[gi];
                    if (swp[gi]) continue;
                    const uint32_t chl = changed_mask(g, cls[gi], ctl[gi]);
                    for (uint32_t q = 0; q < g.a; q++)
                        if (((chl >> g.q[q]) & 1u) && !((needm >> g.q[q]) & 1u)) {
                            needm |= 1u << g.q[q];
                            need.push_back(g.q[q]);
                        }
                    if (need.size() >= nl + nr_max) break;
                }
                if (need.size() > nl + nr_max) need.resize(nl + nr_max);
                needm = 0;
                for (uint32_t q : need) needm |= 1u << q;
                // spare register slots hold needed qubits, which may move to lanes
                for (uint32_t q : need)
                    if ((uint32_t)__builtin_popcount(pend_regs) < nr_max && lay[q] >= nl) pend_regs |= 1u << lay[q];
                std::vector<uint32_t> in, out;
                for (uint32_t q : need)
                    if (lay[q] >= nl && ((pend_regs >> lay[q]) & 1u)) in.push_back(q);
                for (uint32_t pl = 0; pl < nl; pl++)
                    if (!((needm >> inv[pl]) & 1u)) out.push_back(inv[pl]);
                if (rem.empty() && l + 2 <= L) {
                    // at a level's end, the lanes given up go in the order in
                    // which the levels after the next first change their
                    // qubits, earliest first (on QFT-20 and brick-wall trees
                    // faster than lane order: the leaf level of QFT-20 keeps
                    // its lane-controlled phase runs free of register terms)
                    std::vector<uint32_t> first(n, 0xFFFFFFFFu);
                    for (uint32_t gi = cut[l + 2]; gi < cut[L]; gi++) {
                        if (swp[gi]) continue;
                        const uint32_t chl = changed_mask(c->gates[gi], cls[gi], ctl[gi]);
                        for (uint32_t q = 0; q < n; q++)
                            if (((chl >> q) & 1u) && first[q] == 0xFFFFFFFFu) first[q] = gi;
                    }
                    std::stable_sort(out.begin(), out.end(), [&](uint32_t a, uint32_t b) { return first[a] < first[b]; });
                }
                const size_t k = std::min(in.size(), out.size());
                for (size_t i = 0; i < k && pend.size() < 60000; i++) {
                    const uint32_t pr = lay[in[i]], pl = lay[out[i]];
                    PendingGate pg{kNoGate, GC_DENSE2, 0, {pl, pr}};
                    pend.push_back(pg);
                    pend_cost += lane_swap_cost;
                    swap_pos(pl, pr);
                }
            }
            emit();
        }
        lv.pass_count = (uint32_t)p->passes.size() - lv.pass_begin;
        p->levels.push_back(lv);
    }
    p->lay_final = lay;
    {
        // sampling partial sums: chunks of 2^c physically consecutive
        // amplitudes, one partial per block the chunk touches
        const uint32_t cbits = std::min(n, 12u);
        uint32_t cmask = 0;
        for (uint32_t q = p->sample_b; q < n; q++) cmask |= 1u << lay[q];
        const uint32_t kc = (uint32_t)__builtin_popcount(cmask & ((1u << cbits) - 1u));
        p->part_log = n - cbits + kc;
        // partials from the final tile of the last leaf pass
        const tqs::Level &ll = p->levels.back();
        if (!tu.separate_sampling && ll.pass_count > 0) {
            const tqs::PassDesc &pd = p->passes[ll.pass_begin + ll.pass_count - 1];
            uint32_t smask = 0;
            for (uint32_t q = 0; q < p->sample_b; q++) smask |= 1u << lay[q];
            const uint32_t rb = p->reg_bits;
            if (pd.nl == kLaneBits && pd.nr == rb) {
                const uint32_t fold_l = smask & ((1u << kLaneBits) - 1u);
                uint32_t fold_r = 0;
                for (uint32_t i = 0; i < rb; i++)
                    if ((smask >> pd.rq[i]) & 1u) fold_r |= 1u << i;
                const uint32_t nlc = kLaneBits - (uint32_t)__builtin_popcount(fold_l);
                const uint32_t kv = nlc + rb - (uint32_t)__builtin_popcount(fold_r);
                if (kv + 3 <= kLaneBits + rb) {
                    p->samp_tiled = 1;
                    p->samp_psum = fold_l | fold_r << 8 | kv << 16;
                    p->samp_kv = kv;
                    p->samp_nfree = pd.nfree;
                    for (uint32_t t = 0; t < pd.nfree; t++)
                        if ((smask >> pd.fbits[t]) & 1u) p->samp_tfree |= 1u << t;
                    for (uint32_t q = p->sample_b; q < n; q++) {
                        const uint32_t P = lay[q];
                        uint8_t src = 0;
                        if (P < kLaneBits) {
                            src = (uint8_t)(0x80u | (uint32_t)__builtin_popcount(~fold_l & ((1u << P) - 1u)));
                        } else {
                            bool found = false;
                            for (uint32_t i = 0; i < rb && !found; i++)
                                if (pd.rq[i] == P) {
                                    src = (uint8_t)(0x80u | (nlc + (uint32_t)__builtin_popcount(~fold_r & ((1u << i) - 1u))));
                                    found = true;
                                }
                            for (uint32_t t = 0; t < pd.nfree && !found; t++)
                                if (pd.fbits[t] == P) {
                                    src = (uint8_t)t;
                                    found = true;
                                }
                        }
                        p->samp_bsrc[q - p->sample_b] = src;
                    }
                }
            }
        }
    }
    if (p->passes.size() >= (1u << 16)) {
        delete p;
        return fail(TQS_E_UNSUPPORTED, "too many passes (%zu)", p->passes.size());
    }
    for (uint32_t l = 0; l < L; l++)
        p->chunk.push_back((uint32_t)std::min<uint64_t>(p->level_nodes[l], tu.chunk_states));
    if (tu.jit == 1 && prec == TQS_C64 && tu.mfma_min_ops < 1000) fuse_blocks(p, tu.mfma_min_ops);
    *out = p;
    return TQS_OK;
    TQS_GUARD_END
}

// Passes of a plan weighted by the nodes of their level: a run's state reads
// and writes in units of one state, every node computed.
static double weighted_passes(const tqs_plan *p) {
    double w = 0.0;
    for (size_t l = 0; l < p->levels.size(); l++) w += (double)p->level_nodes[l] * p->levels[l].pass_count;
    return w;
}

extern "C" tqs_status tqs_plan_create(const tqs_circuit *c, const tqs_tree *tree, tqs_precision prec,
                                      const tqs_tuning *tuning, tqs_plan **out) {
    TQS_GUARD_BEGIN
    tqs_tuning tu{};
    if (tuning) tu = *tuning;
    if (tu.level_exchange != 0) return plan_create_one(c, tree, prec, &tu, out);
    // default: plan without and with lane exchanges at the levels' ends and
    // keep the exchanges only when they save at least a tenth of the passes
    // weighted by their levels' nodes.  They also change the later levels'
    // layout, which can make their passes slower: on the 20-qubit QFT tree
    // (16, 32, 32) they save 3% of the weighted passes and the leaf pass
    // slows by 2.5%; on the 20-qubit brick-wall tree (8, 8, 16, 16) they save
    // 28% and the run is 9% faster
    tu.level_exchange = 2;
    const tqs_status st = plan_create_one(c, tree, prec, &tu, out);
    if (st != TQS_OK || tree->levels < 2) return st;
    tqs_plan *alt = nullptr;
    tu.level_exchange = 1;
    if (plan_create_one(c, tree, prec, &tu, &alt) != TQS_OK) return TQS_OK;
    if (weighted_passes(alt) <= 0.9 * weighted_passes(*out)) {
        tqs_plan_destroy(*out);
        *out = alt;
    } else {
        tqs_plan_destroy(alt);
    }
    return TQS_OK;
    TQS_GUARD_END
}

namespace tqs {

// Register-only dense ops of full complex64 tiles with five register qubits,
// fused in runs of consecutive ops: U = U_last ... U_first, each op's
// matrix embedded in the 32-dimensional register space (FP64).
void fuse_blocks(tqs_plan *p, uint32_t min_ops) {
    for (uint32_t pi = 0; pi < (uint32_t)p->passes.size(); pi++) {
        const PassDesc &d = p->passes[pi];
        if (d.nr != 5 || d.nl != kLaneBits) continue;
        auto fusable = [&](const OpDesc &o) {
            if (o.kind == OP_DIAGRUN) return false;
            for (uint32_t q = 0; q < o.nq; q++)
                if (o.role[q] != ROLE_REG) return false;
            return true;
        };
        uint32_t oi = d.op_begin;
        const uint32_t oe = d.op_begin + d.op_count;
        while (oi < oe) {
            if (!fusable(p->ops[oi])) {
                oi++;
                continue;
            }
            uint32_t oj = oi;
            while (oj < oe && fusable(p->ops[oj])) oj++;
            if (oj - oi >= min_ops) {
                std::vector<cd> U(32 * 32, cd(0.0, 0.0)), T(32 * 32);
                for (uint32_t r = 0; r < 32; r++) U[r * 32 + r] = cd(1.0, 0.0);
                for (uint32_t k = oi; k < oj; k++) {
                    const OpDesc &o = p->ops[k];
                    const uint32_t nd = 1u << o.nq;
                    uint32_t mask = 0;
                    for (uint32_t q = 0; q < o.nq; q++) mask |= 1u << o.pos[q];
                    auto loc = [&](uint32_t r) {
                        uint32_t x = 0;
                        for (uint32_t q = 0; q < o.nq; q++) x |= ((r >> o.pos[q]) & 1u) << q;
                        return x;
                    };
                    // T = G U, G the op embedded (identity on the other bits)
                    for (uint32_t r = 0; r < 32; r++)
                        for (uint32_t c = 0; c < 32; c++) {
                            cd acc(0.0, 0.0);
                            for (uint32_t b = 0; b < nd; b++) {
                                uint32_t m = r & ~mask;
                                for (uint32_t q = 0; q < o.nq; q++) m |= ((b >> q) & 1u) << o.pos[q];
                                acc += p->mats[o.mat + loc(r) * nd + b] * U[m * 32 + c];
                            }
                            T[r * 32 + c] = acc;
                        }
                    U.swap(T);
                }
                FusedBlock fb;
                fb.pass = pi;
                fb.op_begin = oi;
                fb.op_end = oj;
                fb.mat = (uint32_t)p->mats.size();
                p->mats.insert(p->mats.end(), U.begin(), U.end());
                p->blocks.push_back(fb);
            }
            oi = oj;
        }
    }
}

}  // namespace tqs

extern "C" tqs_status tqs_plan_info(const tqs_plan *p, uint32_t level, uint32_t *passes_level,
                                    uint32_t *passes_total, uint32_t *chunk_states) {
    if (!p) return fail(TQS_E_ARG, "plan is NULL");
    if (level >= p->levels.size()) return fail(TQS_E_ARG, "level %u out of range", level);
    if (passes_level) *passes_level = p->levels[level].pass_count;
    if (passes_total) *passes_total = (uint32_t)p->passes.size();
    if (chunk_states) *chunk_states = p->chunk[level];
    return TQS_OK;
}

extern "C" void tqs_plan_destroy(tqs_plan *p) { delete p; }

// Text description of a plan (see the header for the format).
extern "C" tqs_status tqs_plan_describe(const tqs_plan *p, char *buf, uint64_t cap, uint64_t *len) {
    TQS_GUARD_BEGIN
    if (!p || !len) return fail(TQS_E_ARG, "plan or len is NULL");
    std::string s;
    char tmp[128];
    auto put = [&](const char *fmt, auto... a) {
        std::snprintf(tmp, sizeof tmp, fmt, a...);
        s += tmp;
    };
    put("plan %u %zu %u %zu\n", p->n, p->passes.size(), p->n_gates, p->levels.size());
    s += "layout";
    for (uint32_t q = 0; q < p->n; q++) put(" %u", p->lay_final[q]);
    s += "\n";
    for (uint32_t g = 0; g < p->n_gates; g++)
        put("gate %u %u %u %u %u %u\n", g, p->gate_pass[g], p->gate_pos[g], p->gate_a[g], p->gate_q0[g],
            p->gate_q1[g]);
    for (size_t l = 0; l < p->levels.size(); l++)
        put("level %zu %u %u\n", l, p->levels[l].pass_begin, p->levels[l].pass_count);
    for (size_t pi = 0; pi < p->passes.size(); pi++) {
        const PassDesc &d = p->passes[pi];
        put("pass %zu %u regs", pi, d.op_count);
        for (uint32_t i = 0; i < d.nr; i++) put(" %u", d.rq[i]);
        s += "\n";
        for (uint32_t oi = d.op_begin; oi < d.op_begin + d.op_count; oi++) {
            const OpDesc &o = p->ops[oi];
            if (o.kind == OP_DIAGRUN) {
                put("diag %u %u", o.slot0, o.slot1);
                for (uint32_t k = 0; k < o.ngates; k++) {
                    const DiagGate &dg = p->dgates[o.gates + k];
                    put(" | %u %u %u", dg.nq, dg.phys[0], dg.nq == 2 ? dg.phys[1] : dg.phys[0]);
                    for (uint32_t r = 0; r < (1u << dg.nq); r++)
                        put(" %.17g %.17g", p->mats[dg.d + r].real(), p->mats[dg.d + r].imag());
                }
            } else {
                put("dense %u %u %u %u %u |", o.nq, o.phys[0], o.nq == 2 ? o.phys[1] : o.phys[0], o.slot0,
                    o.slot1);
                const uint32_t nd = 1u << o.nq;
                for (uint32_t r = 0; r < nd * nd; r++)
                    put(" %.17g %.17g", p->mats[o.mat + r].real(), p->mats[o.mat + r].imag());
            }
            s += "\n";
        }
    }
    for (const FusedBlock &fb : p->blocks) put("block %u %u %u\n", fb.pass, fb.op_begin, fb.op_end);
    put("sampling %u %u %u %u %u |", p->samp_tiled, p->samp_kv, p->samp_nfree, p->samp_tfree, p->samp_psum);
    for (uint32_t q = p->sample_b; q < p->n; q++) put(" %u", (uint32_t)p->samp_bsrc[q - p->sample_b]);
    s += "\n";
    *len = s.size() + 1;
    if (buf && cap) {
        const uint64_t k = std::min<uint64_t>(cap - 1, s.size());
        std::memcpy(buf, s.data(), k);
        buf[k] = 0;
    }
    return TQS_OK;
    TQS_GUARD_END
}
