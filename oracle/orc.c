/*
 * Plain CPU oracle for tree-based noisy trajectory simulation (TQSim,
 * arXiv 2203.13892).  TEST INFRASTRUCTURE ONLY: nothing in the product
 * library links, includes or calls this file.  Only the tests, the smoke
 * check and the benchmark's CPU-baseline leg use it.
 *
 * Everything is complex128, one gate at a time, no fusion, no SIMD
 * intrinsics, no blocking.  Each function names the passage of the paper
 * it follows.
 *
 * Conventions (shared with the product only through the written
 * definitions below, never through code):
 *   - bit q of a basis index x is qubit q (little-endian);
 *   - a gate on qubits (q_0, .., q_{a-1}) has a (2^a x 2^a) row-major complex
 *     matrix whose local index bit j is qubit q_j;
 *   - a Pauli code on an a-qubit gate is sum_j c_j 4^j with
 *     c = 0:I, 1:X, 2:Y, 3:Z acting on q_j;
 *   - noise is inserted right after its gate, on that gate's qubits
 *     (Sec. 2.4: noise operators are integrated into the circuit).
 *
 * Random numbers (the paper does not fix a generator): SplitMix64
 * (Steele, Lea, Flood, OOPSLA 2014).  The stream of tree node nu under
 * seed s is SplitMix64 started at state s + nu * 2^32 * gamma, so draw j of
 * node nu is  mix(s + (nu * 2^32 + j + 1) * gamma)  (mod 2^64).
 * A draw becomes a double in [0,1) as (z >> 11) * 2^-53.
 * Per node, in gate order: one uniform u1 per gate; if u1 < p_g (p_g = the
 * sum of the non-identity probabilities in increasing code order) a second
 * uniform u2 picks the code c as the first one whose running sum of
 * probabilities exceeds u2 * p_g (falling back to the largest code with a
 * nonzero probability).  A leaf node then draws one more uniform: its
 * measurement uniform.  With read-out noise (Sec. 4.3, read-out channel:
 * each measured bit flips with its own probability r_q) the leaf then draws
 * n more uniforms v_0 .. v_{n-1}, and bit q of its outcome flips when
 * v_q < r_q.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

typedef struct { double re, im; } cplx;

/* ---------------------------------------------------------------- RNG -- */

/* SplitMix64 output function (published definition). */
static uint64_t sm_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Draw j of node nu's stream. */
uint64_t orc_draw(uint64_t seed, uint64_t nu, uint64_t j) {
    return sm_mix(seed + ((nu << 32) + j + 1) * GAMMA);
}

static double to_unit(uint64_t z) { return (double)(z >> 11) * 0x1.0p-53; }

double orc_uniform(uint64_t seed, uint64_t nu, uint64_t j) {
    return to_unit(orc_draw(seed, nu, j));
}

/* --------------------------------------------------------- tree shape -- */
/* Sec. 3.1: level l (0-based) has prod_{j<=l} A_j nodes; node (l, m) has
 * parent (l-1, m / A_l).  Nodes get global ids level by level. */

static uint64_t level_nodes(const uint64_t *A, int l) {
    uint64_t p = 1;
    for (int j = 0; j <= l; j++) p *= A[j];
    return p;
}

static uint64_t level_offset(const uint64_t *A, int l) {
    uint64_t off = 0;
    for (int j = 0; j < l; j++) off += level_nodes(A, j);
    return off;
}

/* ---------------------------------------------------- noise sampling -- */
/* Sec. 2.4 (pure-state stochastic simulation): each trajectory inserts
 * randomly drawn noise operators after the gates.  Sec. 3.1: every tree node
 * is one instance of its subcircuit with its own noise. */

static int pick_code(const double *pr, int ncodes, double u2) {
    double p = 0.0;
    for (int c = 1; c < ncodes; c++) p += pr[c];
    double t = u2 * p, cum = 0.0;
    for (int c = 1; c < ncodes; c++) {
        cum += pr[c];
        if (t < cum) return c;
    }
    for (int c = ncodes - 1; c >= 1; c--)
        if (pr[c] > 0.0) return c;
    return 0;
}

/* Sample one node: gates [g0, g1).  Writes events if ev_gate != NULL.
 * Returns the number of events; *leaf_u gets the measurement uniform when
 * is_leaf; *j_end (if not NULL) the index of the node's next draw. */
static uint64_t sample_node(uint64_t seed, uint64_t nu, uint64_t g0, uint64_t g1,
                            const int *arity, const double *probs,
                            const int64_t *prob_off, int is_leaf,
                            uint32_t *ev_gate, uint8_t *ev_code, double *leaf_u,
                            uint64_t *j_end) {
    uint64_t j = 0, ne = 0;
    for (uint64_t g = g0; g < g1; g++) {
        double u1 = orc_uniform(seed, nu, j++);
        if (prob_off[g] < 0) continue;
        const double *pr = probs + prob_off[g];
        int ncodes = 1 << (2 * arity[g]);
        double p = 0.0;
        for (int c = 1; c < ncodes; c++) p += pr[c];
        if (u1 < p) {
            double u2 = orc_uniform(seed, nu, j++);
            int c = pick_code(pr, ncodes, u2);
            if (ev_gate) {
                ev_gate[ne] = (uint32_t)g;
                ev_code[ne] = (uint8_t)c;
            }
            ne++;
        }
    }
    if (is_leaf) {
        double u = orc_uniform(seed, nu, j++);
        if (leaf_u) *leaf_u = u;
    }
    if (j_end) *j_end = j;
    return ne;
}

/* Count pass: node_off[nodes+1] (CSR offsets over global node ids). */
int orc_noise_count(uint64_t seed, int levels, const uint64_t *A, const uint64_t *cut,
                    const int *arity, const double *probs, const int64_t *prob_off,
                    uint64_t *node_off) {
    uint64_t nu = 0;
    node_off[0] = 0;
    for (int l = 0; l < levels; l++) {
        uint64_t I = level_nodes(A, l);
        for (uint64_t m = 0; m < I; m++, nu++) {
            uint64_t ne = sample_node(seed, nu, cut[l], cut[l + 1], arity, probs,
                                      prob_off, 0, NULL, NULL, NULL, NULL);
            node_off[nu + 1] = node_off[nu] + ne;
        }
    }
    return 0;
}

/* Fill pass: events and leaf uniforms (leaf_u has prod A entries). */
int orc_noise_fill(uint64_t seed, int levels, const uint64_t *A, const uint64_t *cut,
                   const int *arity, const double *probs, const int64_t *prob_off,
                   const uint64_t *node_off, uint32_t *ev_gate, uint8_t *ev_code,
                   double *leaf_u) {
    uint64_t nu = 0;
    for (int l = 0; l < levels; l++) {
        uint64_t I = level_nodes(A, l);
        int is_leaf = (l == levels - 1);
        for (uint64_t m = 0; m < I; m++, nu++) {
            sample_node(seed, nu, cut[l], cut[l + 1], arity, probs, prob_off, is_leaf,
                        ev_gate + node_off[nu], ev_code + node_off[nu],
                        is_leaf ? &leaf_u[m] : NULL, NULL);
        }
    }
    return 0;
}

/* Read-out flips: leaf_flip[m] gets bit q set when leaf m's draw v_q is
 * below r[q] (the n draws after its measurement uniform). */
int orc_readout_fill(uint64_t seed, int levels, const uint64_t *A, const uint64_t *cut,
                     const int *arity, const double *probs, const int64_t *prob_off,
                     int n, const double *r, uint32_t *leaf_flip) {
    uint64_t nu = 0;
    for (int l = 0; l < levels - 1; l++) nu += level_nodes(A, l);
    const int L = levels - 1;
    uint64_t I = level_nodes(A, L);
    for (uint64_t m = 0; m < I; m++, nu++) {
        uint64_t j = 0;
        sample_node(seed, nu, cut[L], cut[L + 1], arity, probs, prob_off, 1, NULL, NULL, NULL, &j);
        uint32_t f = 0;
        for (int q = 0; q < n; q++)
            if (orc_uniform(seed, nu, j++) < r[q]) f |= 1u << q;
        leaf_flip[m] = f;
    }
    return 0;
}

/* ------------------------------------------------------ state vector -- */
/* Sec. 2.2: the state is a vector of 2^n amplitudes and a gate is a matrix
 * multiplied into it.  Written for an arbitrary a-qubit gate: for every
 * assignment of the other qubits, gather the 2^a amplitudes, multiply by the
 * matrix, scatter. */

/* The gate on the index range [x0, x1) of the other qubits' assignments. */
static void apply_gate_range(double *psi_d, int a, const int *q, const double *mat_d,
                             uint64_t x0, uint64_t x1) {
    cplx *psi = (cplx *)psi_d;
    const cplx *M = (const cplx *)mat_d;
    int k = 1 << a;
    uint64_t mask = 0;
    for (int j = 0; j < a; j++) mask |= 1ULL << q[j];
    cplx in[4], out[4];
    uint64_t idx[4];
    for (uint64_t x = x0; x < x1; x++) {
        if (x & mask) continue; /* x enumerates the other qubits */
        for (int l = 0; l < k; l++) {
            uint64_t y = x;
            for (int j = 0; j < a; j++)
                if ((l >> j) & 1) y |= 1ULL << q[j];
            idx[l] = y;
            in[l] = psi[y];
        }
        for (int r = 0; r < k; r++) {
            double re = 0.0, im = 0.0;
            for (int c = 0; c < k; c++) {
                cplx m = M[r * k + c];
                re += m.re * in[c].re - m.im * in[c].im;
                im += m.re * in[c].im + m.im * in[c].re;
            }
            out[r].re = re;
            out[r].im = im;
        }
        for (int l = 0; l < k; l++) psi[idx[l]] = out[l];
    }
}

void orc_apply_gate(int n, double *psi_d, int a, const int *q, const double *mat_d) {
    apply_gate_range(psi_d, a, q, mat_d, 0, 1ULL << n);
}

/* The same gate with the index loop split into `parts` contiguous ranges
 * run by threads.  Every group of amplitudes is still read, multiplied and
 * written by the same expression, exactly once, so the result is identical
 * to orc_apply_gate's; this only lets spare threads help a leaf when there
 * are fewer leaves than threads. */
typedef struct {
    double *psi;
    int a;
    const int *q;
    const double *mat;
    uint64_t x0, x1;
} range_t;

static void *range_worker(void *arg) {
    const range_t *R = (const range_t *)arg;
    apply_gate_range(R->psi, R->a, R->q, R->mat, R->x0, R->x1);
    return NULL;
}

static void apply_gate_split(int n, double *psi, int a, const int *q, const double *mat, int parts) {
    uint64_t dim = 1ULL << n;
    if (parts <= 1 || dim < 4096) {
        apply_gate_range(psi, a, q, mat, 0, dim);
        return;
    }
    if (parts > 64) parts = 64;
    range_t R[64];
    pthread_t th[64];
    int started[64];
    for (int t = 0; t < parts; t++) {
        R[t].psi = psi; R[t].a = a; R[t].q = q; R[t].mat = mat;
        R[t].x0 = dim * (uint64_t)t / (uint64_t)parts;
        R[t].x1 = dim * (uint64_t)(t + 1) / (uint64_t)parts;
        started[t] = t > 0 && pthread_create(&th[t], NULL, range_worker, &R[t]) == 0;
    }
    /* this thread takes range 0, and any range whose thread did not start */
    range_worker(&R[0]);
    for (int t = 1; t < parts; t++)
        if (!started[t]) range_worker(&R[t]);
    for (int t = 1; t < parts; t++)
        if (started[t]) pthread_join(th[t], NULL);
}

/* The one-qubit Pauli matrices I, X, Y, Z. */
static const double PAULI[4][8] = {
    {1, 0, 0, 0, 0, 0, 1, 0},
    {0, 0, 1, 0, 1, 0, 0, 0},
    {0, 0, 0, -1, 0, 1, 0, 0},
    {1, 0, 0, 0, 0, 0, -1, 0},
};

/* A Pauli noise operator on the gate's qubits, applied as its one-qubit
 * factors (plain matrix products). */
static void apply_pauli_split(int n, double *psi, int a, const int *q, int code, int parts) {
    for (int j = 0; j < a; j++) {
        int c = (code >> (2 * j)) & 3;
        if (c) apply_gate_split(n, psi, 1, &q[j], PAULI[c], parts);
    }
}

void orc_apply_pauli(int n, double *psi, int a, const int *q, int code) {
    apply_pauli_split(n, psi, a, q, code, 1);
}

/* Sec. 2.2: an outcome is sampled from the final state.  Inverse CDF in
 * FP64 over the index order: x = min{x : sum_{y<=x} |psi_y|^2 > u * T}. */
uint64_t orc_sample_state(int n, const double *psi_d, double u) {
    const cplx *psi = (const cplx *)psi_d;
    uint64_t dim = 1ULL << n;
    double T = 0.0;
    for (uint64_t x = 0; x < dim; x++) T += psi[x].re * psi[x].re + psi[x].im * psi[x].im;
    double t = u * T, cum = 0.0;
    for (uint64_t x = 0; x < dim; x++) {
        cum += psi[x].re * psi[x].re + psi[x].im * psi[x].im;
        if (cum > t) return x;
    }
    for (uint64_t x = dim; x-- > 0;)
        if (psi[x].re * psi[x].re + psi[x].im * psi[x].im > 0.0) return x;
    return 0;
}

/* --------------------------------------------------------- trajectories -- */

typedef struct {
    int n, levels;
    const int *arity, *qubits;
    const double *mats;
    const int64_t *mat_off;
    const uint64_t *A, *cut;
    const uint64_t *node_off;
    const uint32_t *ev_gate;
    const uint8_t *ev_code;
    const double *leaf_u;
    const uint64_t *leaves;
    uint64_t n_leaves;
    uint64_t *outcomes;
    double *states;
    int nthreads, tid;
    int parts; /* threads per gate application (1 unless leaves < threads) */
} job_t;

/* One leaf = one full trajectory, computed from scratch (no reuse): the
 * leaf's ancestors supply the noise of every subcircuit (Sec. 3.1). */
static void run_leaf(const job_t *J, uint64_t lam, double *psi) {
    uint64_t dim = 1ULL << J->n;
    memset(psi, 0, dim * 2 * sizeof(double));
    psi[0] = 1.0;
    for (int l = 0; l < J->levels; l++) {
        uint64_t below = 1;
        for (int j = l + 1; j < J->levels; j++) below *= J->A[j];
        uint64_t nu = level_offset(J->A, l) + lam / below;
        uint64_t e = J->node_off[nu], e1 = J->node_off[nu + 1];
        for (uint64_t g = J->cut[l]; g < J->cut[l + 1]; g++) {
            const int *q = J->qubits + 2 * g;
            apply_gate_split(J->n, psi, J->arity[g], q, J->mats + J->mat_off[g], J->parts);
            while (e < e1 && J->ev_gate[e] == g) {
                apply_pauli_split(J->n, psi, J->arity[g], q, J->ev_code[e], J->parts);
                e++;
            }
        }
    }
}

static void *worker(void *arg) {
    job_t *J = (job_t *)arg;
    uint64_t dim = 1ULL << J->n;
    double *psi = (double *)malloc(dim * 2 * sizeof(double));
    if (!psi) return (void *)1;
    for (uint64_t i = (uint64_t)J->tid; i < J->n_leaves; i += (uint64_t)J->nthreads) {
        uint64_t lam = J->leaves[i];
        run_leaf(J, lam, psi);
        if (J->outcomes) J->outcomes[i] = orc_sample_state(J->n, psi, J->leaf_u[lam]);
        if (J->states) memcpy(J->states + i * dim * 2, psi, dim * 2 * sizeof(double));
    }
    free(psi);
    return NULL;
}

/* Simulate the listed leaves independently (threads over leaves; with
 * fewer leaves than threads, the spare threads split each gate's loop). */
int orc_run_leaves(int n, const int *arity, const int *qubits, const double *mats,
                   const int64_t *mat_off, int levels, const uint64_t *A,
                   const uint64_t *cut, const uint64_t *node_off, const uint32_t *ev_gate,
                   const uint8_t *ev_code, const double *leaf_u, const uint64_t *leaves,
                   uint64_t n_leaves, uint64_t *outcomes, double *states, int nthreads) {
    if (nthreads < 1) nthreads = 1;
    int parts = 1;
    if ((uint64_t)nthreads > n_leaves) {
        parts = n_leaves ? nthreads / (int)n_leaves : 1;
        nthreads = n_leaves ? (int)n_leaves : 1;
    }
    job_t *jobs = (job_t *)calloc((size_t)nthreads, sizeof(job_t));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !th) return -1;
    int rc = 0, started = 0;
    for (int t = 0; t < nthreads; t++) {
        job_t *J = &jobs[t];
        J->n = n; J->levels = levels; J->arity = arity; J->qubits = qubits;
        J->mats = mats; J->mat_off = mat_off; J->A = A; J->cut = cut;
        J->node_off = node_off; J->ev_gate = ev_gate; J->ev_code = ev_code;
        J->leaf_u = leaf_u; J->leaves = leaves; J->n_leaves = n_leaves;
        J->outcomes = outcomes; J->states = states; J->nthreads = nthreads; J->tid = t;
        J->parts = parts;
        if (pthread_create(&th[t], NULL, worker, J)) {
            rc = -1;
            break;
        }
        started++;
    }
    for (int t = 0; t < started; t++) {
        void *r = NULL;
        pthread_join(th[t], &r);
        if (r) rc = -1;
    }
    free(jobs);
    free(th);
    return rc;
}
