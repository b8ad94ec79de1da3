// Internal declarations of the tqsim library (host planner + HIP executor).
#pragma once

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "tqsim.h"

namespace tqs {

using cd = std::complex<double>;

constexpr uint32_t kMaxQubits = 30;
constexpr uint32_t kMaxTile = 12;        // qubits per workgroup tile (LDS <= 64 KiB)
constexpr uint32_t kMinContig = 6;       // contiguous low qubits per tile run (512 B at c64)
constexpr uint32_t kThreads = 256;       // threads per pass workgroup
constexpr uint8_t kNotLocal = 0xFF;

// ------------------------------------------------------------- errors --
tqs_status fail(tqs_status st, const char *fmt, ...);
void clear_error();

// ------------------------------------------------------------ circuit --
struct Gate {
    uint32_t a = 1;          // arity 1 or 2
    uint32_t q[2] = {0, 0};  // logical = physical qubits
    cd m[16];                // (2^a)^2 row-major
    bool noisy = false;
    double pr[16] = {0};     // 4^a Pauli-code probabilities
    double p_err = 0.0;      // sum of the non-identity probabilities, code order
};

}  // namespace tqs

struct tqs_circuit {
    uint32_t n = 0;
    std::vector<tqs::Gate> gates;
};

struct tqs_noise {
    uint32_t n_gates = 0;
    std::vector<uint64_t> arity;
    std::vector<uint32_t> cut;
    uint64_t n_nodes = 0, n_leaves = 0;
    std::vector<uint64_t> node_off;
    std::vector<uint32_t> ev_gate;
    std::vector<uint8_t> ev_code;
    std::vector<double> leaf_u;
};

namespace tqs {

// Op kinds applied inside a pass tile.
enum OpKind : uint8_t {
    OP_DENSE1 = 0,  // one-qubit matrix on a staged qubit
    OP_DENSE2 = 1,  // two-qubit matrix on two staged qubits
    OP_DIAG = 2,    // diagonal 1q/2q gate, qubits anywhere
    OP_CTRL = 3,    // 2q gate block-diagonal in one qubit (anywhere), dense in a staged one
};

// Device-side op descriptor (12 bytes).
struct OpDesc {
    uint8_t kind;
    uint8_t nq;
    uint8_t loc[2];   // tile-local bit of each gate qubit or kNotLocal
    uint8_t phys[2];  // physical qubit of each gate qubit
    uint8_t ctrl;     // OP_CTRL: which gate qubit (0/1) is block-diagonal
    uint8_t pad;
    uint32_t mat;     // offset in complex entries into the plan's matrix table
};

// Device-side pass descriptor.
struct PassDesc {
    uint32_t op_begin, op_count;
    uint32_t m;            // tile qubits
    uint32_t c;            // contiguous low qubits 0..c-1
    uint32_t nh;           // staged high qubits (m - c)
    uint32_t nfree;        // n - m tile-index qubits
    uint8_t hbits[16];     // physical qubit of local bit c + i
    uint8_t fbits[32];     // physical qubit of tile-index bit i
};

struct Level {
    uint32_t pass_begin = 0, pass_count = 0;
    uint32_t g0 = 0, g1 = 0;
};

}  // namespace tqs

struct tqs_plan {
    ~tqs_plan();
    uint32_t n = 0;
    tqs_precision prec = TQS_C64;
    tqs_tuning tune{};
    std::vector<uint64_t> arity;
    std::vector<uint32_t> cut;
    std::vector<uint64_t> level_nodes;   // I_l
    std::vector<uint64_t> level_offset;  // global id of node (l, 0)
    uint64_t n_nodes = 0, n_leaves = 0;
    uint32_t n_gates = 0;
    std::vector<tqs::Level> levels;
    std::vector<tqs::PassDesc> passes;
    std::vector<tqs::OpDesc> ops;
    std::vector<tqs::cd> mats;
    // where an event after gate g takes effect: pass (global index) and op
    // position inside that pass
    std::vector<uint32_t> gate_pass, gate_pos;
    std::vector<uint32_t> gate_q0, gate_q1, gate_a;  // physical qubits per gate
    std::vector<uint32_t> chunk;  // live states per level
    uint32_t sample_b = 12;
    std::vector<void *> events;  // hipEvent_t pool for run statistics
};

namespace tqs {
// planner helpers shared with the executor
uint64_t level_nodes(const std::vector<uint64_t> &A, uint32_t l);
tqs_status validate_tree(const tqs_tree *t, uint32_t n_gates, std::vector<uint64_t> *A,
                         std::vector<uint32_t> *cut);
}  // namespace tqs
