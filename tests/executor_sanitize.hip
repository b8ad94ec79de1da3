// The executor's host-side steps (per-node frames and events, the chunk
// schedule with shared states, the workspace layout and the metadata
// packing) driven on random circuits, trees, tunings and noise under
// AddressSanitizer and UndefinedBehaviorSanitizer.  Built with hipcc by
// tests/test_host.py, the sanitizers on the host code only; no HIP call is
// made and no kernel launched.
#include "device.hip"

#include <cstdlib>
#include <random>

static int fails = 0;
#define CHECK(c)                                                            \
    do {                                                                    \
        if (!(c)) {                                                         \
            std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            fails++;                                                        \
        }                                                                   \
    } while (0)

// the schedule's invariants for the subtrees [first, last)
static void check_schedule(const tqs_plan *p, const HostMeta *hm, uint64_t first, uint64_t last,
                           const std::vector<Task> &tasks, const std::vector<uint32_t> &sched) {
    const uint32_t L = (uint32_t)p->arity.size();
    std::vector<uint64_t> seen_nodes(L, 0);
    // the state slot each node was last given (tasks run depth first, so a
    // parent's entry is the one its children read)
    std::vector<uint32_t> slot_of_node(p->n_nodes, 0xFFFFFFFFu);
    for (const Task &t : tasks) {
        CHECK(t.level < L);
        CHECK(t.ccount >= 1 && t.ccount <= t.count && t.ccount <= p->chunk[t.level]);
        CHECK(t.sched + 3ull * t.count + 3ull * t.ccount <= sched.size());
        seen_nodes[t.level] += t.count;
        for (uint32_t i = 0; i < t.count; i++) {
            const uint32_t node = sched[t.node_ids() + i];
            CHECK(node == p->level_offset[t.level] + t.first + i);
            const uint32_t r = sched[t.rep_of() + i];
            CHECK(r < t.ccount);
            if (r >= t.ccount) continue;
            CHECK(sched[t.slot_of() + i] == sched[t.cdst() + r]);
            const uint32_t cn = sched[t.cnode() + r];
            // the state it uses is computed from its own parent's state
            const uint64_t m = t.first + i;
            const uint32_t from = t.level == 0 ? kInit
                                               : slot_of_node[p->level_offset[t.level - 1] + m / p->arity[t.level]];
            CHECK(sched[t.csrc() + r] == from);
            if (!hm) {
                CHECK(r == i && cn == node);
                continue;
            }
            // a node shares the state of a computed node with its history
            CHECK(same_history(*hm, cn, node));
            // and no two computed states of a task have the same source and history
            for (uint32_t j = 0; j < r; j++)
                CHECK(!(sched[t.csrc() + j] == sched[t.csrc() + r] &&
                        same_history(*hm, sched[t.cnode() + j], sched[t.cnode() + r])));
        }
        for (uint32_t i = 0; i < t.count; i++) slot_of_node[sched[t.node_ids() + i]] = sched[t.slot_of() + i];
    }
    uint64_t want = last - first;
    for (uint32_t l = 0; l < L; l++) {
        if (l > 0) want *= p->arity[l];
        CHECK(seen_nodes[l] == want);
    }
}

int main(int argc, char **argv) {
    const int cases = argc > 1 ? std::atoi(argv[1]) : 200;
    std::mt19937_64 g(777);
    // the key table: entries with equal keys are all visited
    {
        SeenTable t;
        t.reset(40);
        for (uint32_t v = 0; v < 20; v++) t.insert(v % 3 == 0 ? 42u : 1000u + v, v);
        for (uint32_t v = 0; v < 20; v++) {
            const uint64_t k = v % 3 == 0 ? 42u : 1000u + v;
            CHECK(t.find(k, [&](uint32_t x) { return x == v; }) == (int64_t)v);
        }
        CHECK(t.find(7u, [](uint32_t) { return true; }) == -1);
        t.reset(40);
        CHECK(t.find(42u, [](uint32_t) { return true; }) == -1);
    }
    int runs = 0;
    for (int it = 0; it < cases; it++) {
        const uint32_t n = 1 + g() % 14;
        tqs_circuit *c = nullptr;
        if (tqs_circuit_create(n, &c) != TQS_OK) return 1;
        const uint32_t G = 1 + g() % 60;
        for (uint32_t k = 0; k < G; k++) {
            const uint32_t a = (n >= 2 && g() % 2) ? 2 : 1;
            uint32_t q[2] = {(uint32_t)(g() % n), 0};
            if (a == 2) do q[1] = (uint32_t)(g() % n); while (q[1] == q[0]);
            const int d = 1 << a;
            std::vector<double> m(2 * d * d, 0.0);
            const double ph = std::uniform_real_distribution<double>(0, 6.3)(g);
            if (g() % 2) {
                // diagonal
                for (int r = 0; r < d; r++) {
                    m[2 * (r * d + r)] = std::cos(ph * r);
                    m[2 * (r * d + r) + 1] = std::sin(ph * r);
                }
            } else {
                // a real rotation on the first qubit (identity on the second)
                for (int r = 0; r < d; r += 2) {
                    m[2 * (r * d + r)] = std::cos(ph);
                    m[2 * (r * d + r + 1)] = -std::sin(ph);
                    m[2 * ((r + 1) * d + r)] = std::sin(ph);
                    m[2 * ((r + 1) * d + r + 1)] = std::cos(ph);
                }
            }
            std::vector<double> pr(1u << (2 * a), 0.0);
            const double pe = std::uniform_real_distribution<double>(0, 0.4)(g);
            pr[0] = 1 - pe;
            for (size_t i = 1; i < pr.size(); i++) pr[i] = pe / (pr.size() - 1);
            if (tqs_circuit_add_gate(c, a, q, m.data(), g() % 4 ? pr.data() : nullptr) != TQS_OK) return 2;
        }
        const uint32_t L = 1 + g() % std::min<uint32_t>(4, G);
        std::vector<uint64_t> A(L);
        for (auto &x : A) x = 1 + g() % 6;
        std::vector<uint32_t> cut(L + 1, 0);
        for (uint32_t l = 1; l < L; l++)
            cut[l] = cut[l - 1] + 1 + g() % std::max<uint32_t>(1, (G - cut[l - 1]) / (L - l + 1));
        cut[L] = G;
        tqs_tree tree{L, A.data(), cut.data()};
        tqs_tuning tu{};
        if (g() % 2) tu.max_ops_per_pass = 1 + g() % 30;
        if (g() % 2) tu.chunk_states = 1 + g() % 9;
        if (g() % 2) tu.sample_block_log = 8 + g() % 5;
        tu.separate_sampling = g() % 2;
        tu.level_exchange = g() % 3;
        // specialised kernels: routing, frame tables and code generation
        // (host side; nothing is compiled or loaded)
        tu.jit = 1 + g() % 2;
        if (g() % 2) tu.mfma_min_ops = 1 + g() % 8;
        tqs_plan *p = nullptr;
        if (tqs_plan_create(c, &tree, g() % 2 ? TQS_C64 : TQS_C128, &tu, &p) != TQS_OK) {
            tqs_circuit_destroy(c);
            continue;
        }
        if (tu.jit == 1) {
            uint64_t len = 0;
            CHECK(tqs_plan_jit_source(p, nullptr, 0, &len) == TQS_OK && len > 0);
            std::vector<char> src(len);
            CHECK(tqs_plan_jit_source(p, src.data(), len, &len) == TQS_OK && src[len - 1] == 0);
        }
        tqs_noise *nz = nullptr;
        if (tqs_noise_sample(c, &tree, g(), &nz) != TQS_OK) return 3;
        if (check_noise(p, nz) != TQS_OK) return 4;
        HostMeta hm;
        build_meta(p, nz, &hm);
        CHECK(hm.ev_off[p->n_nodes] == nz->ev_gate.size());
        for (uint64_t nu = 0; nu < p->n_nodes; nu++) {
            CHECK(hm.ev_eff[nu] <= hm.ev_off[nu + 1] - hm.ev_off[nu]);
            for (uint32_t e = hm.ev_off[nu] + 1; e < hm.ev_off[nu + 1]; e++) CHECK(hm.ev_pos[e - 1] <= hm.ev_pos[e]);
        }
        const uint64_t first = g() % A[0], last = first + 1 + g() % (A[0] - first);
        for (int merge = 0; merge < 2; merge++) {
            std::vector<Task> tasks;
            std::vector<uint32_t> sched;
            const uint64_t per = p->n_leaves / A[0];
            Layout Ly0 = make_layout(p, nz->ev_gate.size(), (last - first) * per, 0);
            build_schedule(p, first, last, &tasks, &sched, Ly0.slot_base, merge ? &hm : nullptr);
            check_schedule(p, merge ? &hm : nullptr, first, last, tasks, sched);
            const size_t sched0 = sched.size();
            std::vector<std::vector<Route>> routes;
            FrameTables ftab;
            route_passes(p, hm, tasks, &sched, &routes, &ftab);
            CHECK(routes.size() == tasks.size());
            CHECK(ftab.tab.size() <= table_bound(p));
            for (size_t ti = 0; ti < tasks.size(); ti++) {
                const Task &t = tasks[ti];
                CHECK(routes[ti].size() == p->levels[t.level].pass_count);
                if (p->tune.jit != 1)
                    for (const Route &r : routes[ti]) CHECK(r.n_jit == 0 && r.perm == Route::kNoPerm);
                for (const Route &r : routes[ti]) {
                    CHECK(r.n_jit <= t.ccount);
                    if (r.perm == Route::kNoPerm) continue;
                    // a permutation of the chunk's computed states
                    CHECK(r.perm >= sched0 && r.perm + t.ccount <= sched.size());
                    std::vector<char> seen(t.ccount, 0);
                    for (uint32_t c = 0; c < t.ccount && r.perm + t.ccount <= sched.size(); c++) {
                        const uint32_t v = sched[r.perm + c];
                        CHECK(v < t.ccount && !seen[v]);
                        if (v < t.ccount) seen[v] = 1;
                    }
                }
            }
            for (uint64_t nu = 0; nu < p->n_nodes; nu++) {
                const uint32_t o = ftab.ct_off[nu];
                if (o == 0xFFFFFFFFu) continue;
                CHECK(o < sched.size());
                const uint32_t cnt = o < sched.size() ? sched[o] : 0;
                CHECK(o + 1 + 2ull * cnt <= sched.size());
                for (uint32_t i = 0; i < cnt && o + 1 + 2ull * cnt <= sched.size(); i++) {
                    CHECK(sched[o + 1 + 2 * i] < p->passes.size());
                    CHECK(sched[o + 2 + 2 * i] < ftab.tab.size());
                }
            }
            Layout Ly = make_layout(p, nz->ev_gate.size(), (last - first) * per, sched.size(), 0, ~0ull,
                                    ftab.tab.size());
            CHECK(sched.size() - sched0 <= route_bound(p));
            // within what tqs_workspace_bytes promises: for any list, and for
            // this list (whole runs share states unless the tuning says not to)
            uint64_t bound = 0;
            CHECK(tqs_workspace_bytes(p, nullptr, &bound) == TQS_OK && Ly.total <= bound);
            if (merge != p->tune.no_merge) CHECK(tqs_workspace_bytes(p, nz, &bound) == TQS_OK && Ly.total <= bound);
            std::vector<unsigned char> hb(Ly.off_sums - Ly.off_meta, 0);
            if (p->prec == TQS_C64) pack_meta<float>(p, nz, hm, sched, Ly, hb.data(), Ly.off_meta, &ftab);
            else pack_meta<double>(p, nz, hm, sched, Ly, hb.data(), Ly.off_meta, &ftab);
            runs++;
        }
        tqs_noise_destroy(nz);
        tqs_plan_destroy(p);
        tqs_circuit_destroy(c);
    }
    std::printf("cases %d runs %d fails %d\n", cases, runs, fails);
    return fails ? 5 : 0;
}
