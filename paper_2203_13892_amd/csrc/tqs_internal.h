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
constexpr uint32_t kLaneBits = 6;        // 64 lanes per wave
constexpr uint32_t kMaxRegBits = 6;      // register qubits per tile (64 amplitudes per lane)
constexpr uint32_t kThreads = 256;       // threads per sampling workgroup
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
    std::vector<double> readout;  // per-qubit read-out flip probability (empty: none)
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
    std::vector<uint32_t> leaf_flip;  // read-out flip mask per leaf (empty: none)
};

namespace tqs {

// Op kinds applied inside a pass tile.
enum OpKind : uint8_t {
    OP_DENSE1 = 0,   // 2x2 on one staged qubit, optionally selected by a control qubit
    OP_DENSE2 = 1,   // 4x4 on two staged qubits
    OP_DIAGRUN = 2,  // a run of consecutive diagonal gates, qubits anywhere
};

// Where a qubit sits in a pass tile.  A workgroup is one wave; lane L holds
// the amplitudes with low bits L (lane qubits = physical 0..nl-1) and
// register index j over the register qubits; the remaining (free) qubits
// are fixed per tile.
enum Role : uint8_t { ROLE_LANE = 0, ROLE_REG = 1, ROLE_FIXED = 2 };

// Device-side op descriptor.
struct OpDesc {
    uint8_t kind;
    uint8_t nq;        // gate arity
    uint8_t role[2];   // per gate qubit
    uint8_t pos[2];    // lane bit, register bit, or physical qubit (fixed)
    uint8_t phys[2];   // physical qubit per gate qubit (frame bits)
    uint8_t tq;        // OP_DENSE1 with nq == 2: gate qubit that is the target
    uint8_t real;      // DENSE1/DENSE2: every matrix entry is real
    uint8_t has_t;     // DIAGRUN: some gates act on register qubits only (the table)
    uint8_t lam_mask;  // DIAGRUN: register bits that fixed+register or lane+register terms touch
    uint16_t slot0, slot1;  // gate slots [slot0, slot1) of the pass covered by the op
    uint32_t mat;      // DENSE1/DENSE2: matrix offset; DIAGRUN: table offset (2^nr entries)
    uint32_t terms;    // DIAGRUN: first term touching a non-register qubit
    uint32_t tmask;    // DIAGRUN: register-table entries that are not exactly 1
    uint32_t gates;    // DIAGRUN: first per-gate record (slow path)
    uint32_t ngates;
    // DIAGRUN term groups, stored in this order: fixed-only terms, then
    // fixed+register terms by register bit, then lane terms (lane / lane+lane /
    // lane+fixed), then lane+register terms by register bit
    uint16_t n_fix;
    uint16_t n_lane;
    uint16_t n_fixreg[kMaxRegBits];
    uint16_t n_lanereg[kMaxRegBits];
};

// A diagonal gate of a run that touches a lane or fixed qubit: its phases
// theta(r) = arg d(r) / (2 pi) as 64-bit fixed-point turns.
struct DiagTerm {
    uint8_t nq;
    uint8_t role[2];
    uint8_t pos[2];
    uint8_t phys[2];
    uint8_t k;  // index of its gate in the run (255: 255 or later)
    uint64_t th[4];
};

// A diagonal gate of a run, for gate-by-gate application.
struct DiagGate {
    uint8_t nq;
    uint8_t role[2];
    uint8_t pos[2];
    uint8_t phys[2];
    uint8_t pad;
    uint32_t d;  // offset of its 2^nq diagonal entries
};

// Device-side pass descriptor.
struct PassDesc {
    uint32_t op_begin, op_count;
    uint8_t nl;          // lane qubits (physical 0..nl-1)
    uint8_t nr;          // register qubits
    uint8_t nfree;       // tile-index qubits
    uint8_t has_d2;      // contains OP_DENSE2 ops
    uint8_t rq[8];       // physical qubit of register bit i
    uint8_t fbits[32];   // physical qubit of tile-index bit i
    // the pass's slices of the matrix and term tables (staged in LDS)
    uint32_t mat_begin, mat_count;
    uint32_t term_begin, term_count;
};

constexpr uint32_t kPassLdsBytes = 16384;  // LDS budget for one pass's staged data

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
    std::vector<tqs::DiagTerm> terms;
    std::vector<tqs::DiagGate> dgates;
    uint32_t reg_bits = 6;
    // where an event after gate g takes effect: pass (global index) and the
    // gate slot inside that pass after which it acts
    std::vector<uint32_t> gate_pass, gate_pos;
    std::vector<uint32_t> gate_q0, gate_q1, gate_a;  // physical qubits per gate
    // physical position of each logical qubit once the last level has run
    // (swap gates and the planner's lane exchanges permute positions)
    std::vector<uint32_t> lay_final;
    uint32_t part_log = 0;  // log2 of the sampling partial sums per state
    // sampling partials written by the last pass of the leaf level (when
    // its final tile is full and leaves at least 8 amplitudes per partial):
    // lane bits summed | register bits summed << 8 | pattern bits << 16,
    // tile-index bits, tile-index bits inside a block, and per block-index
    // bit its source: 0x80 | pattern bit, or the tile-index bit
    uint32_t samp_tiled = 0, samp_psum = 0, samp_kv = 0, samp_nfree = 0, samp_tfree = 0;
    uint8_t samp_bsrc[32] = {0};
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
