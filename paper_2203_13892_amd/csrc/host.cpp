// Host side of tqsim: circuit IR, noise insertion list, Dynamic Circuit
// Partition, pass planner, histogram.  No device code here.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "tqs_internal.h"

namespace tqs {

static thread_local std::string g_err = "no error";

tqs_status fail(tqs_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

void clear_error() { g_err = "no error"; }

uint64_t level_nodes(const std::vector<uint64_t> &A, uint32_t l) {
    uint64_t p = 1;
    for (uint32_t j = 0; j <= l; j++) p *= A[j];
    return p;
}

// Sec. 3.1: arities >= 1, cuts strictly increasing from 0 to G.
tqs_status validate_tree(const tqs_tree *t, uint32_t n_gates, std::vector<uint64_t> *A,
                         std::vector<uint32_t> *cut) {
    if (!t || !t->arity || !t->cut) return fail(TQS_E_ARG, "tree, arity or cut is NULL");
    if (t->levels < 1 || t->levels > 64)
        return fail(TQS_E_SHAPE, "levels must be in 1..64 (got %u)", t->levels);
    if (t->cut[0] != 0 || t->cut[t->levels] != n_gates)
        return fail(TQS_E_SHAPE, "cut must start at 0 and end at the gate count %u", n_gates);
    __uint128_t leaves = 1, nodes = 0;
    for (uint32_t l = 0; l < t->levels; l++) {
        if (t->arity[l] < 1) return fail(TQS_E_SHAPE, "arity[%u] is 0", l);
        if (t->cut[l + 1] <= t->cut[l])
            return fail(TQS_E_SHAPE, "cuts must be strictly increasing (cut[%u]=%u, cut[%u]=%u)",
                        l, t->cut[l], l + 1, t->cut[l + 1]);
        leaves *= t->arity[l];
        nodes += leaves;
        if (nodes > (((__uint128_t)1) << 32))
            return fail(TQS_E_SHAPE, "tree has more than 2^32 nodes");
    }
    if (A) A->assign(t->arity, t->arity + t->levels);
    if (cut) cut->assign(t->cut, t->cut + t->levels + 1);
    return TQS_OK;
}

// ------------------------------------------------------------- SplitMix64 --
// Steele, Lea & Flood (2014).  Node nu's stream starts at state
// seed + nu * 2^32 * gamma; draw j is the output after j + 1 increments.
static inline uint64_t splitmix_out(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

struct NodeStream {
    uint64_t state;
    NodeStream(uint64_t seed, uint64_t nu) : state(seed + (nu << 32) * 0x9E3779B97F4A7C15ULL) {}
    double next() {
        state += 0x9E3779B97F4A7C15ULL;
        return (double)(splitmix_out(state) >> 11) * 0x1.0p-53;
    }
};

}  // namespace tqs

using namespace tqs;

#define TQS_GUARD_BEGIN try {
#define TQS_GUARD_END                                                            \
    }                                                                            \
    catch (const std::bad_alloc &) {                                             \
        return fail(TQS_E_OOM, "host allocation failed");                        \
    }                                                                            \
    catch (...) {                                                                \
        return fail(TQS_E_ARG, "unexpected exception");                          \
    }

extern "C" {

const char *tqs_last_error(void) { return g_err.c_str(); }

const char *tqs_version(void) { return "tqsim-gfx950 1.0"; }

// ------------------------------------------------------------------ circuit --

tqs_status tqs_circuit_create(uint32_t n_qubits, tqs_circuit **out) {
    TQS_GUARD_BEGIN
    if (!out) return fail(TQS_E_ARG, "out is NULL");
    *out = nullptr;
    if (n_qubits < 1 || n_qubits > kMaxQubits)
        return fail(TQS_E_UNSUPPORTED, "n_qubits must be in 1..%u (got %u)", kMaxQubits, n_qubits);
    tqs_circuit *c = new tqs_circuit;
    c->n = n_qubits;
    *out = c;
    return TQS_OK;
    TQS_GUARD_END
}

void tqs_circuit_destroy(tqs_circuit *c) { delete c; }

tqs_status tqs_circuit_add_gate(tqs_circuit *c, uint32_t arity, const uint32_t *qubits,
                                const double *mat, const double *pauli) {
    TQS_GUARD_BEGIN
    if (!c || !qubits || !mat) return fail(TQS_E_ARG, "circuit, qubits or mat is NULL");
    if (arity != 1 && arity != 2) return fail(TQS_E_ARG, "arity must be 1 or 2 (got %u)", arity);
    Gate g;
    g.a = arity;
    for (uint32_t j = 0; j < arity; j++) {
        if (qubits[j] >= c->n)
            return fail(TQS_E_ARG, "qubit %u out of range (n=%u)", qubits[j], c->n);
        g.q[j] = qubits[j];
    }
    if (arity == 2 && g.q[0] == g.q[1]) return fail(TQS_E_ARG, "two-qubit gate on one qubit");
    const int k = 1 << arity;
    for (int i = 0; i < k * k; i++) {
        if (!std::isfinite(mat[2 * i]) || !std::isfinite(mat[2 * i + 1]))
            return fail(TQS_E_ARG, "matrix entry %d is not finite", i);
        g.m[i] = cd(mat[2 * i], mat[2 * i + 1]);
    }
    // unitarity: M M^dagger = I within 1e-9
    for (int r = 0; r < k; r++)
        for (int s = 0; s < k; s++) {
            cd acc = 0;
            for (int t = 0; t < k; t++) acc += g.m[r * k + t] * std::conj(g.m[s * k + t]);
            if (std::abs(acc - cd(r == s ? 1.0 : 0.0, 0.0)) > 1e-9)
                return fail(TQS_E_ARG, "gate matrix is not unitary (entry %d,%d off by %.3g)", r, s,
                            std::abs(acc - cd(r == s ? 1.0 : 0.0, 0.0)));
        }
    if (pauli) {
        const int nc = 1 << (2 * arity);
        double tot = 0;
        for (int i = 0; i < nc; i++) {
            if (!(pauli[i] >= 0.0) || !std::isfinite(pauli[i]))
                return fail(TQS_E_ARG, "Pauli probability %d is negative or not finite", i);
            g.pr[i] = pauli[i];
            tot += pauli[i];
        }
        if (std::fabs(tot - 1.0) > 1e-9) return fail(TQS_E_ARG, "Pauli probabilities sum to %.12g", tot);
        double p = 0.0;
        for (int i = 1; i < nc; i++) p += g.pr[i];
        g.p_err = p;
        g.noisy = true;
    }
    c->gates.push_back(g);
    return TQS_OK;
    TQS_GUARD_END
}

tqs_status tqs_circuit_set_depolarizing(tqs_circuit *c, double p1, double p2) {
    if (!c) return fail(TQS_E_ARG, "circuit is NULL");
    if (!(p1 >= 0.0 && p1 <= 1.0) || !(p2 >= 0.0 && p2 <= 1.0))
        return fail(TQS_E_ARG, "depolarizing probabilities must be in [0, 1]");
    for (Gate &g : c->gates) {
        const double p = g.a == 1 ? p1 : p2;
        const int nc = 1 << (2 * g.a);
        std::fill(g.pr, g.pr + 16, 0.0);
        if (p <= 0.0) {
            g.noisy = false;
            g.p_err = 0.0;
            continue;
        }
        g.pr[0] = 1.0 - p;
        for (int i = 1; i < nc; i++) g.pr[i] = p / (nc - 1);
        double s = 0.0;
        for (int i = 1; i < nc; i++) s += g.pr[i];
        g.p_err = s;
        g.noisy = true;
    }
    return TQS_OK;
}

tqs_status tqs_circuit_set_readout(tqs_circuit *c, const double *p_flip) {
    if (!c) return fail(TQS_E_ARG, "circuit is NULL");
    if (!p_flip) {
        c->readout.clear();
        return TQS_OK;
    }
    for (uint32_t q = 0; q < c->n; q++)
        if (!(p_flip[q] >= 0.0 && p_flip[q] <= 1.0))
            return fail(TQS_E_ARG, "read-out probability of qubit %u not in [0, 1]", q);
    c->readout.assign(p_flip, p_flip + c->n);
    return TQS_OK;
}

tqs_status tqs_circuit_info(const tqs_circuit *c, uint32_t *n_qubits, uint32_t *n_gates) {
    if (!c) return fail(TQS_E_ARG, "circuit is NULL");
    if (n_qubits) *n_qubits = c->n;
    if (n_gates) *n_gates = (uint32_t)c->gates.size();
    return TQS_OK;
}

// -------------------------------------------------------------------- DCP --

tqs_status tqs_dcp(const tqs_circuit *c, uint64_t shots, double z, double eps, double copy_cost,
                   uint32_t max_levels, uint32_t *levels, uint64_t *arity, uint32_t *cut) {
    TQS_GUARD_BEGIN
    if (!c || !levels || !arity || !cut) return fail(TQS_E_ARG, "NULL argument");
    if (shots < 1) return fail(TQS_E_ARG, "shots must be >= 1");
    if (!(z > 0) || !(eps > 0) || !(copy_cost >= 0) || !std::isfinite(copy_cost))
        return fail(TQS_E_ARG, "z and eps must be > 0, copy_cost >= 0");
    if (max_levels < 1) return fail(TQS_E_ARG, "max_levels must be >= 1");
    const uint64_t G = c->gates.size();
    if (G == 0) return fail(TQS_E_ARG, "empty circuit");
    const uint64_t N = shots;
    // first subcircuit: the fewest gates that amortise one state copy
    const uint64_t L0 = std::max<uint64_t>(1, (uint64_t)std::ceil(copy_cost));
    auto per_shot = [&]() {
        *levels = 1;
        arity[0] = N;
        cut[0] = 0;
        cut[1] = (uint32_t)G;
        return TQS_OK;
    };
    if (L0 >= G) return per_shot();
    // first-subcircuit error rate 1 - prod(1 - e_i)
    double prod = 1.0;
    for (uint64_t i = 0; i < L0; i++) prod *= (1.0 - c->gates[i].p_err);
    const double ph = 1.0 - prod;
    // sample-size bound for A_0
    const double n0 = z * z * ph * (1.0 - ph) / (eps * eps);
    const double a0 = n0 / (1.0 + n0 / (double)N);
    uint64_t A0min = (uint64_t)std::ceil(a0);
    A0min = std::min<uint64_t>(std::max<uint64_t>(A0min, 1), N);
    // floor((N / A0min)^(1/k)) computed exactly: largest a with a^k * A0min <= N
    auto root_floor = [&](uint32_t k) -> uint64_t {
        const long double r = (long double)N / (long double)A0min;
        uint64_t a = (uint64_t)std::floor(std::pow(r, 1.0L / k)) + 2;
        while (a > 0) {
            __uint128_t p = A0min;
            bool over = false;
            for (uint32_t i = 0; i < k && !over; i++) {
                p *= a;
                if (p > N) over = true;
            }
            if (!over) break;
            a--;
        }
        return a;
    };
    uint32_t k_shots = 0;
    while (k_shots < 63 && root_floor(k_shots + 1) >= 2) k_shots++;
    const uint64_t k_gates = (uint64_t)std::floor((double)(G - L0) / std::max(1.0, copy_cost));
    uint64_t k = std::min<uint64_t>(k_shots, k_gates);
    k = std::min<uint64_t>(k, max_levels - 1);
    if (k < 1) return per_shot();
    const uint64_t Ar = root_floor((uint32_t)k);
    uint64_t Ark = 1;
    for (uint64_t i = 0; i < k; i++) Ark *= Ar;
    const uint64_t A0 = (N + Ark - 1) / Ark;
    *levels = (uint32_t)(k + 1);
    arity[0] = A0;
    for (uint64_t i = 1; i <= k; i++) arity[i] = Ar;
    const uint64_t rest = G - L0;
    cut[0] = 0;
    cut[1] = (uint32_t)L0;
    for (uint64_t i = 0; i < k; i++)
        cut[i + 2] = cut[i + 1] + (uint32_t)(rest / k + (i < rest % k ? 1 : 0));
    return TQS_OK;
    TQS_GUARD_END
}

// ------------------------------------------------------------------ noise --

tqs_status tqs_noise_sample(const tqs_circuit *c, const tqs_tree *tree, uint64_t seed,
                            tqs_noise **out) {
    TQS_GUARD_BEGIN
    if (!c || !out) return fail(TQS_E_ARG, "circuit or out is NULL");
    *out = nullptr;
    std::vector<uint64_t> A;
    std::vector<uint32_t> cut;
    tqs_status st = validate_tree(tree, (uint32_t)c->gates.size(), &A, &cut);
    if (st) return st;
    tqs_noise *nz = new tqs_noise;
    nz->n_gates = (uint32_t)c->gates.size();
    nz->arity = A;
    nz->cut = cut;
    const uint32_t L = (uint32_t)A.size();
    uint64_t nodes = 0;
    for (uint32_t l = 0; l < L; l++) nodes += level_nodes(A, l);
    nz->n_nodes = nodes;
    nz->n_leaves = level_nodes(A, L - 1);
    nz->node_off.assign(nodes + 1, 0);
    nz->leaf_u.assign(nz->n_leaves, 0.0);
    if (!c->readout.empty()) nz->leaf_flip.assign(nz->n_leaves, 0);
    uint64_t nu = 0;
    for (uint32_t l = 0; l < L; l++) {
        const uint64_t I = level_nodes(A, l);
        const bool leaf = (l == L - 1);
        for (uint64_t m = 0; m < I; m++, nu++) {
            NodeStream rs(seed, nu);
            for (uint32_t g = cut[l]; g < cut[l + 1]; g++) {
                const double u1 = rs.next();
                const Gate &G = c->gates[g];
                if (!G.noisy) continue;
                if (u1 < G.p_err) {
                    const double u2 = rs.next();
                    const int nc = 1 << (2 * G.a);
                    const double t = u2 * G.p_err;
                    double cum = 0.0;
                    int code = 0;
                    for (int k = 1; k < nc; k++) {
                        cum += G.pr[k];
                        if (t < cum) {
                            code = k;
                            break;
                        }
                    }
                    if (!code)
                        for (int k = nc - 1; k >= 1; k--)
                            if (G.pr[k] > 0.0) {
                                code = k;
                                break;
                            }
                    nz->ev_gate.push_back(g);
                    nz->ev_code.push_back((uint8_t)code);
                }
            }
            if (leaf) {
                nz->leaf_u[m] = rs.next();
                if (!c->readout.empty()) {
                    uint32_t f = 0;
                    for (uint32_t q = 0; q < c->n; q++)
                        if (rs.next() < c->readout[q]) f |= 1u << q;
                    nz->leaf_flip[m] = f;
                }
            }
            nz->node_off[nu + 1] = nz->ev_gate.size();
        }
    }
    *out = nz;
    return TQS_OK;
    TQS_GUARD_END
}

tqs_status tqs_noise_import(const tqs_circuit *c, const tqs_tree *tree, const uint64_t *node_off,
                            const uint32_t *ev_gate, const uint8_t *ev_code, const double *leaf_u,
                            tqs_noise **out) {
    TQS_GUARD_BEGIN
    if (!c || !out || !node_off || !leaf_u) return fail(TQS_E_ARG, "NULL argument");
    *out = nullptr;
    std::vector<uint64_t> A;
    std::vector<uint32_t> cut;
    tqs_status st = validate_tree(tree, (uint32_t)c->gates.size(), &A, &cut);
    if (st) return st;
    const uint32_t L = (uint32_t)A.size();
    uint64_t nodes = 0;
    for (uint32_t l = 0; l < L; l++) nodes += level_nodes(A, l);
    const uint64_t leaves = level_nodes(A, L - 1);
    if (node_off[0] != 0) return fail(TQS_E_ARG, "node_off[0] must be 0");
    const uint64_t ne = node_off[nodes];
    if (ne && (!ev_gate || !ev_code)) return fail(TQS_E_ARG, "events given without arrays");
    uint64_t nu = 0;
    for (uint32_t l = 0; l < L; l++) {
        const uint64_t I = level_nodes(A, l);
        for (uint64_t m = 0; m < I; m++, nu++) {
            if (node_off[nu + 1] < node_off[nu]) return fail(TQS_E_ARG, "node_off not monotone");
            // before any event of this node is read: its range must lie
            // inside the list's declared length node_off[nodes]
            if (node_off[nu + 1] > ne)
                return fail(TQS_E_ARG, "node_off[%llu] = %llu beyond node_off[%llu] = %llu",
                            (unsigned long long)(nu + 1), (unsigned long long)node_off[nu + 1],
                            (unsigned long long)nodes, (unsigned long long)ne);
            int64_t prev = -1;
            for (uint64_t e = node_off[nu]; e < node_off[nu + 1]; e++) {
                const uint32_t g = ev_gate[e];
                if (g < cut[l] || g >= cut[l + 1])
                    return fail(TQS_E_ARG, "event gate %u outside node %llu's subcircuit", g,
                                (unsigned long long)nu);
                if ((int64_t)g <= prev) return fail(TQS_E_ARG, "events not sorted by gate");
                prev = g;
                const int nc = 1 << (2 * c->gates[g].a);
                if (ev_code[e] == 0 || ev_code[e] >= nc)
                    return fail(TQS_E_ARG, "event code %u invalid for gate %u", ev_code[e], g);
            }
        }
    }
    for (uint64_t i = 0; i < leaves; i++)
        if (!(leaf_u[i] >= 0.0 && leaf_u[i] < 1.0)) return fail(TQS_E_ARG, "leaf_u[%llu] not in [0,1)",
                                                                (unsigned long long)i);
    tqs_noise *nz = new tqs_noise;
    nz->n_gates = (uint32_t)c->gates.size();
    nz->arity = A;
    nz->cut = cut;
    nz->n_nodes = nodes;
    nz->n_leaves = leaves;
    nz->node_off.assign(node_off, node_off + nodes + 1);
    nz->ev_gate.assign(ev_gate, ev_gate + ne);
    nz->ev_code.assign(ev_code, ev_code + ne);
    nz->leaf_u.assign(leaf_u, leaf_u + leaves);
    *out = nz;
    return TQS_OK;
    TQS_GUARD_END
}

tqs_status tqs_noise_view(const tqs_noise *nz, const uint64_t **node_off, const uint32_t **ev_gate,
                          const uint8_t **ev_code, const double **leaf_u, uint64_t *n_nodes,
                          uint64_t *n_leaves) {
    if (!nz) return fail(TQS_E_ARG, "noise is NULL");
    if (node_off) *node_off = nz->node_off.data();
    if (ev_gate) *ev_gate = nz->ev_gate.data();
    if (ev_code) *ev_code = nz->ev_code.data();
    if (leaf_u) *leaf_u = nz->leaf_u.data();
    if (n_nodes) *n_nodes = nz->n_nodes;
    if (n_leaves) *n_leaves = nz->n_leaves;
    return TQS_OK;
}

tqs_status tqs_noise_set_flips(tqs_noise *nz, const uint32_t *leaf_flip) {
    TQS_GUARD_BEGIN
    if (!nz) return fail(TQS_E_ARG, "noise is NULL");
    if (!leaf_flip) nz->leaf_flip.clear();
    else nz->leaf_flip.assign(leaf_flip, leaf_flip + nz->n_leaves);
    return TQS_OK;
    TQS_GUARD_END
}

tqs_status tqs_noise_flips(const tqs_noise *nz, const uint32_t **leaf_flip) {
    if (!nz || !leaf_flip) return fail(TQS_E_ARG, "noise or leaf_flip is NULL");
    *leaf_flip = nz->leaf_flip.empty() ? nullptr : nz->leaf_flip.data();
    return TQS_OK;
}

void tqs_noise_destroy(tqs_noise *nz) { delete nz; }

}  // extern "C"

// -------------------------------------------------------------- histogram --

extern "C" tqs_status tqs_histogram(const uint64_t *outcomes, uint64_t n, uint64_t *values,
                                    uint64_t *counts, uint64_t *n_unique) {
    TQS_GUARD_BEGIN
    if (!n_unique || (n && (!outcomes || !values || !counts))) return fail(TQS_E_ARG, "NULL argument");
    std::vector<uint64_t> v(outcomes, outcomes + n);
    std::sort(v.begin(), v.end());
    uint64_t u = 0;
    for (uint64_t i = 0; i < n;) {
        uint64_t j = i;
        while (j < n && v[j] == v[i]) j++;
        values[u] = v[i];
        counts[u] = j - i;
        u++;
        i = j;
    }
    *n_unique = u;
    return TQS_OK;
    TQS_GUARD_END
}
