// Internal declarations of the tqsim library (host planner + HIP executor).
#pragma once

#include <complex>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "tqsim.h"
#include "device_types.h"

namespace tqs {

using cd = std::complex<double>;

constexpr uint32_t kMaxQubits = 30;
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


struct Level {
    uint32_t pass_begin = 0, pass_count = 0;
    uint32_t g0 = 0, g1 = 0;
};

// Consecutive dense ops [op_begin, op_end) of a pass on its five register
// qubits, fused into one 32x32 unitary (mats[mat..mat+1024), row-major over
// the register index) that the specialised kernel applies with MFMA.
struct FusedBlock {
    uint32_t pass, op_begin, op_end, mat;
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
    // host side of the runs in flight (tqs_run_start to tqs_run_finish): two
    // slots, each with pinned buffers for the metadata upload and the
    // outcome download (so neither copy waits for the host) and its own
    // hipEvent_t pool for run statistics
    struct RunSlot {
        void *meta = nullptr;
        uint64_t meta_cap = 0;
        void *out = nullptr;
        uint64_t out_cap = 0;
        std::vector<void *> events;
        bool busy = false;
    };
    RunSlot slots[2];
    std::mutex slot_mu;
    // plan-specialised pass kernels (jit.cpp): code object, the module
    // loaded on jit_device, one function per pass (NULL: generic kernel)
    std::vector<tqs::FusedBlock> blocks;  // sorted by pass, then op
    std::vector<char> jit_code;
    void *jit_module = nullptr;
    int jit_device = -1;
    std::vector<void *> jit_fn;
};

namespace tqs {
// A phase run of a pass, for routing nodes to the specialised kernels.
struct JitRun {
    uint32_t s0, s1, ngates;
    uint32_t ro_first, ro_last;  // register-only gates' index span (first > last: none)
    uint32_t regmask;            // physical positions of the pass's register qubits
    uint32_t op;                 // the run's op index
};
// A fused block's slots: events at keys in (first, last] fall between its ops.
struct JitBlock {
    uint32_t first, last;
};
// How a pass's specialised kernel takes a node.
enum JitFit { JIT_NO = 0, JIT_YES = 1, JIT_TABLES = 2 /* with its own frame tables */ };
// Frame tables of one node for pass pi: every table run of the pass, in
// order, 2^nr entries each, with the node's frames at each register-only
// gate applied.  pos/dx/n: the node's events; fx0: its X frame at node start.
void jit_frame_tables(const tqs_plan *p, uint32_t pi, uint32_t fx0, const uint32_t *pos, const uint32_t *dx,
                      uint32_t n, std::vector<cd> *out);
// Table entries of pass pi for one node (0 when the pass has no table run).
uint32_t jit_table_entries(const tqs_plan *p, uint32_t pi);
bool jit_pass_supported(const tqs_plan *p, uint32_t pi);
std::string jit_source(const tqs_plan *p);
tqs_status jit_compile(tqs_plan *p);
tqs_status jit_prepare(tqs_plan *p);
void jit_release(tqs_plan *p);
void jit_runs(const tqs_plan *p, std::vector<std::vector<JitRun>> *runs,
              std::vector<std::vector<JitBlock>> *blocks);
JitFit jit_fit(const std::vector<JitRun> &runs, const std::vector<JitBlock> &blocks, uint32_t pi,
              const uint32_t *pos, const uint32_t *dx, uint32_t n);
// Fuse the register-only dense runs of a complex64 plan (plan creation).
void fuse_blocks(tqs_plan *p, uint32_t min_ops);

// planner helpers shared with the executor
uint64_t level_nodes(const std::vector<uint64_t> &A, uint32_t l);
tqs_status validate_tree(const tqs_tree *t, uint32_t n_gates, std::vector<uint64_t> *A,
                         std::vector<uint32_t> *cut);
}  // namespace tqs
