// Host-side planner, noise sampler, DCP and histogram driven on random
// inputs under AddressSanitizer and UndefinedBehaviorSanitizer (built with
// g++ by tests/test_host.py; no GPU code is linked).
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "tqs_internal.h"

// the executor (device code) owns the plan's event pool; none is created here
tqs_plan::~tqs_plan() {}

static std::vector<double> haar(std::mt19937_64 &g, int d) {
    // a random unitary from QR of a Gaussian matrix (Gram-Schmidt), interleaved re/im
    std::normal_distribution<double> N(0.0, 1.0);
    std::vector<std::complex<double>> m(d * d);
    for (auto &z : m) z = {N(g), N(g)};
    for (int c = 0; c < d; c++) {
        for (int p = 0; p < c; p++) {
            std::complex<double> dot = 0;
            for (int r = 0; r < d; r++) dot += std::conj(m[r * d + p]) * m[r * d + c];
            for (int r = 0; r < d; r++) m[r * d + c] -= dot * m[r * d + p];
        }
        double nrm = 0;
        for (int r = 0; r < d; r++) nrm += std::norm(m[r * d + c]);
        nrm = std::sqrt(nrm);
        for (int r = 0; r < d; r++) m[r * d + c] /= nrm;
    }
    std::vector<double> out(2 * d * d);
    for (int i = 0; i < d * d; i++) {
        out[2 * i] = m[i].real();
        out[2 * i + 1] = m[i].imag();
    }
    return out;
}

int main(int argc, char **argv) {
    const int cases = argc > 1 ? std::atoi(argv[1]) : 200;
    std::mt19937_64 g(12345);
    int planned = 0, refused = 0;
    for (int it = 0; it < cases; it++) {
        const uint32_t n = 1 + g() % 20;
        tqs_circuit *c = nullptr;
        if (tqs_circuit_create(n, &c) != TQS_OK) return 1;
        const uint32_t G = 1 + g() % 80;
        for (uint32_t k = 0; k < G; k++) {
            const uint32_t a = (n >= 2 && g() % 2) ? 2 : 1;
            uint32_t q[2] = {(uint32_t)(g() % n), 0};
            if (a == 2) do q[1] = (uint32_t)(g() % n); while (q[1] == q[0]);
            std::vector<double> m;
            if (g() % 4 == 0) {
                // diagonal phase gate
                const int d = 1 << a;
                m.assign(2 * d * d, 0.0);
                for (int r = 0; r < d; r++) {
                    const double ph = std::uniform_real_distribution<double>(0, 6.3)(g);
                    m[2 * (r * d + r)] = std::cos(ph);
                    m[2 * (r * d + r) + 1] = std::sin(ph);
                }
            } else {
                m = haar(g, 1 << a);
            }
            std::vector<double> pr(1u << (2 * a), 0.0);
            const double p = std::uniform_real_distribution<double>(0, 0.3)(g);
            pr[0] = 1 - p;
            for (size_t i = 1; i < pr.size(); i++) pr[i] = p / (pr.size() - 1);
            if (tqs_circuit_add_gate(c, a, q, m.data(), g() % 3 ? pr.data() : nullptr) != TQS_OK) return 2;
        }
        if (g() % 3 == 0) {
            std::vector<double> r(n);
            for (auto &x : r) x = std::uniform_real_distribution<double>(0, 0.5)(g);
            tqs_circuit_set_readout(c, r.data());
        }
        // a random tree (sometimes invalid)
        const uint32_t L = 1 + g() % std::min<uint32_t>(4, G);
        std::vector<uint64_t> A(L);
        for (auto &x : A) x = 1 + g() % 6;
        std::vector<uint32_t> cut(L + 1, 0);
        for (uint32_t l = 1; l < L; l++) cut[l] = cut[l - 1] + 1 + g() % std::max<uint32_t>(1, (G - cut[l - 1]) / (L - l + 1));
        cut[L] = G;
        if (g() % 10 == 0 && L > 1) cut[1] = cut[0];  // not strictly increasing
        tqs_tree tree{L, A.data(), cut.data()};
        tqs_tuning tu{};
        if (g() % 2) tu.tile_qubits = 10 + g() % 2;
        if (g() % 2) tu.max_ops_per_pass = 1 + g() % 50;
        if (g() % 2) tu.chunk_states = 1 + g() % 7;
        if (g() % 2) tu.sample_block_log = 8 + g() % 9;
        if (g() % 2) tu.pass_cost = 50 + g() % 1000;
        tu.no_merge = g() % 2;
        tu.separate_sampling = g() % 2;
        tu.level_exchange = g() % 3;
        tqs_plan *p = nullptr;
        const tqs_precision prec = g() % 2 ? TQS_C64 : TQS_C128;
        if (tqs_plan_create(c, &tree, prec, &tu, &p) == TQS_OK) {
            planned++;
            uint64_t len = 0;
            tqs_plan_describe(p, nullptr, 0, &len);
            std::vector<char> buf(len);
            tqs_plan_describe(p, buf.data(), len, &len);
            uint32_t pl = 0, pt = 0, cs = 0;
            tqs_plan_info(p, 0, &pl, &pt, &cs);
            tqs_noise *nz = nullptr;
            if (tqs_noise_sample(c, &tree, g(), &nz) == TQS_OK) {
                const uint64_t *off = nullptr;
                const uint32_t *eg = nullptr;
                const uint8_t *ec = nullptr;
                const double *lu = nullptr;
                uint64_t nn = 0, nl = 0;
                tqs_noise_view(nz, &off, &eg, &ec, &lu, &nn, &nl);
                // re-import the same list, then a corrupted one
                tqs_noise *nz2 = nullptr;
                if (tqs_noise_import(c, &tree, off, eg, ec, lu, &nz2) != TQS_OK) return 3;
                if (off[nn] > 0) {
                    std::vector<uint8_t> bad(ec, ec + off[nn]);
                    bad[0] = 0;  // identity code is not an event
                    tqs_noise *nz3 = nullptr;
                    if (tqs_noise_import(c, &tree, off, eg, bad.data(), lu, &nz3) == TQS_OK) return 4;
                    refused++;
                }
                if (nn > 1) {
                    // an offset that overshoots the list's length
                    // node_off[nodes] while the event arrays hold exactly
                    // that many: refused before any event is read
                    std::vector<uint64_t> off2(off, off + nn + 1);
                    const uint64_t k = 1 + g() % (nn - 1);
                    off2[k] = off[nn] + 1 + g() % 7;
                    std::vector<uint32_t> eg2(eg, eg + off[nn]);
                    std::vector<uint8_t> ec2(ec, ec + off[nn]);
                    tqs_noise *nz4 = nullptr;
                    if (tqs_noise_import(c, &tree, off2.data(), eg2.data(), ec2.data(), lu, &nz4) == TQS_OK)
                        return 5;
                    refused++;
                }
                std::vector<uint32_t> fl(nl, 1u);
                tqs_noise_set_flips(nz2, fl.data());
                const uint32_t *fv = nullptr;
                tqs_noise_flips(nz2, &fv);
                tqs_noise_destroy(nz2);
                tqs_noise_destroy(nz);
            }
            tqs_plan_destroy(p);
        } else {
            refused++;
        }
        // DCP and histogram on the same circuit
        uint32_t lv = 0;
        uint64_t dA[8];
        uint32_t dc[9];
        tqs_dcp(c, 1 + g() % 40000, 1.96, 0.01, std::uniform_real_distribution<double>(0, 40)(g), 8, &lv, dA, dc);
        std::vector<uint64_t> outc(1 + g() % 500);
        for (auto &x : outc) x = g() % 64;
        std::vector<uint64_t> vals(outc.size()), cnts(outc.size());
        uint64_t nu = 0;
        tqs_histogram(outc.data(), outc.size(), vals.data(), cnts.data(), &nu);
        tqs_circuit_destroy(c);
    }
    std::printf("cases %d planned %d refused %d\n", cases, planned, refused);
    return 0;
}
