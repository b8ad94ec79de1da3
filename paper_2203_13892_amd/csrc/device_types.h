// Plan records read by the pass kernels (host planner and device code,
// including kernels compiled at run time): plain structs of fixed-width
// integers, no library headers.
#pragma once

namespace tqs {

constexpr uint32_t kLaneBits = 6;    // 64 lanes per wave
constexpr uint32_t kMaxRegBits = 6;  // register qubits per tile (64 amplitudes per lane)

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

}  // namespace tqs
