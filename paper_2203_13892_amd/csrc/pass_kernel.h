// Gate-apply pass kernel for gfx950: one wave per workgroup, one tile of
// one trajectory per wave, the whole tile held in registers.
//
// Tile layout: lane L (0..63) holds the amplitudes whose physical qubits
// 0..nl-1 spell L, register index j (0..2^RB-1) spells the register qubits
// rq[0..nr-1], and the free qubits are fixed by the tile index.  Each
// register index is one fully coalesced wave load / store (64 consecutive
// amplitudes).  Gates on register qubits are in-register butterflies, gates
// on lane qubits exchange partners with cross-lane shuffles, diagonal gates
// need no exchange at all.  Nothing goes through LDS and the wave never
// waits on a barrier; every amplitude is read once and written once.
//
// Noise is carried by the trajectory's Pauli frame (x, z): a gate G acts on
// the stored state as F^dagger G F, i.e. G[r ^ x][c ^ x] (-1)^{z.r + z.c} on
// the gate's local indices.  Frame updates are events placed between gate
// slots of the pass.
#pragma once

#include <cstddef>
#include <type_traits>
#include <utility>

namespace tqs {

// Read-only pass data (descriptors, matrices, phase terms, noise metadata)
// is read through constant-address-space pointers: the compiler may then use
// scalar loads for wave-uniform addresses, since nothing the kernel writes
// can alias them.
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using kptr = const __attribute__((address_space(4))) T *;
#else
template <typename T>
using kptr = const T *;  // host pass: kernel bodies are only parsed there
#endif
template <typename T>
__device__ __forceinline__ kptr<T> kconst(const T *p) {
    return (kptr<T>)p;
}

// Copy of a read-only record, dword by dword (wave-uniform address: scalar
// loads).
template <typename T>
__device__ __forceinline__ T kload(kptr<T> p) {
    static_assert(sizeof(T) % 4 == 0, "record of whole dwords");
    T out;
    uint32_t *d = reinterpret_cast<uint32_t *>(&out);
    const kptr<uint32_t> w = (kptr<uint32_t>)p;
#pragma unroll
    for (uint32_t i = 0; i < sizeof(T) / 4; i++) d[i] = w[i];
    return out;
}

// A wave-uniform value, kept in a scalar register: a per-lane select between
// two such values stays a register select (and is not turned into a per-lane
// load from a selected address).
__device__ __forceinline__ uint32_t uni(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)x);
}
__device__ __forceinline__ uint64_t uni(uint64_t x) {
    const uint32_t lo = uni((uint32_t)x), hi = uni((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// A phase term read as whole dwords (scalar loads cannot read bytes): its
// arity, the role of its second qubit, its physical qubits and its four
// phases in the accumulator width A.
template <typename A>
struct TermU {
    uint32_t nq, role1, phys0, phys1, k;
    A th[4];
};
template <typename A>
__device__ __forceinline__ TermU<A> load_term(kptr<DiagTerm> p) {
    static_assert(sizeof(DiagTerm) == 40, "phase term layout");
    const kptr<uint32_t> w = (kptr<uint32_t>)p;
    const uint32_t w0 = uni(w[0]), w1 = uni(w[1]);
    TermU<A> t;
    t.nq = w0 & 0xFFu;
    t.role1 = (w0 >> 16) & 0xFFu;
    t.phys0 = (w1 >> 8) & 0xFFu;
    t.phys1 = (w1 >> 16) & 0xFFu;
    t.k = (w1 >> 24) & 0xFFu;
#pragma unroll
    for (int r = 0; r < 4; r++) {
        if constexpr (sizeof(A) == 4) t.th[r] = uni(w[2 + 2 * r]);
        else t.th[r] = uni((uint64_t)w[2 + 2 * r] | ((uint64_t)w[3 + 2 * r] << 32));
    }
    return t;
}

// One pass over `count` states of one plan (a segment of a launch).
template <typename R>
struct PassArgs {
    cplx<R> *states;
    uint64_t slot_amps;
    const uint32_t *node_ids;
    const uint32_t *src_slot;
    const uint32_t *dst_slot;
    uint32_t count;
    uint32_t work;      // count * tiles (unpadded)
    uint32_t pass_key;
    uint32_t wg_begin;  // first workgroup of this segment in the launch
    const PassDesc *pass;
    const OpDesc *ops;
    const cplx<R> *mats;
    const DiagTerm *terms;
    const DiagGate *dgates;
    NodeMeta meta;
    // sampling partials of the written states (last pass of the leaf level;
    // NULL otherwise): per state and tile, the FP64 mass of each pattern of
    // the block-index bits that vary inside the tile
    double *part;
    uint32_t psum;  // lane bits summed (bits 0-7), register bits summed (8-15), pattern bits (16-23)
    uint32_t pad;
};

// A launch: one segment passed by value, or a table of segments (passes
// of different plans, for batches) in device memory, sorted by wg_begin.
template <typename R>
struct PassLaunch {
    PassArgs<R> one;
    const PassArgs<R> *segs;
    uint32_t nseg;   // 0: `one` is the launch
    uint32_t total;  // workgroups with work
};

template <typename R>
__device__ __forceinline__ cplx<R> csel(bool c, cplx<R> a, cplx<R> b) {
    return c ? a : b;
}

template <typename R>
__device__ __forceinline__ cplx<R> shfl_xor_c(cplx<R> v, uint32_t mask) {
    return {__shfl_xor(v.re, (int)mask), __shfl_xor(v.im, (int)mask)};
}

// Real-coefficient products (the matrix entry's imaginary part is zero).
template <typename R>
__device__ __forceinline__ cplx<R> rmul(cplx<R> m, cplx<R> x) {
    return {m.re * x.re, m.re * x.im};
}
template <typename R>
__device__ __forceinline__ cplx<R> rmac(cplx<R> acc, cplx<R> m, cplx<R> x) {
    return {acc.re + m.re * x.re, acc.im + m.re * x.im};
}

// Bounds how much independent work the scheduler hoists ahead of its use
// (cross-lane exchanges, products): each hoisted result holds registers until
// consumed, and the tile already fills most of them.  A fence after every
// 4th register index.
template <int J>
__device__ __forceinline__ void shuffle_fence() {
    if constexpr ((J & 3) == 3) __builtin_amdgcn_sched_barrier(0);
}

// e^{2 pi i t} for fixed-point turns t, from arithmetic only (no table, so
// no memory latency inside a phase run): t = q/4 + r with q the nearest
// quarter turn and |r| <= 1/8 turn; the Taylor series of cos and sin at
// x = 2 pi r (|x| <= pi/4) to x^10 / x^9 in single precision (truncation
// below 2e-9) and to x^18 / x^17 in double (below 1e-19); then the quarter
// turn i^q swaps and negates the two parts.
__device__ __forceinline__ cplx<float> expi_turns(uint32_t t) {
    const uint32_t q = ((t + (1u << 29)) >> 30) & 3u;
    const int32_t r = (int32_t)(t - (q << 30));
    const float x = (float)r * 1.4629180792671596e-09f;  // 2 pi / 2^32
    const float x2 = x * x;
    float ps = 1.0f / 362880.0f;
    ps = ps * x2 - 1.0f / 5040.0f;
    ps = ps * x2 + 1.0f / 120.0f;
    ps = ps * x2 - 1.0f / 6.0f;
    ps = ps * x2 + 1.0f;
    float pc = -1.0f / 3628800.0f;
    pc = pc * x2 + 1.0f / 40320.0f;
    pc = pc * x2 - 1.0f / 720.0f;
    pc = pc * x2 + 1.0f / 24.0f;
    pc = pc * x2 - 0.5f;
    pc = pc * x2 + 1.0f;
    const float sn = x * ps;
    const bool odd = (q & 1u) != 0;
    cplx<float> e = {odd ? sn : pc, odd ? pc : sn};
    return cneg_parts(e, ((q + 1u) >> 1) & 1u, q >> 1);
}
__device__ __forceinline__ cplx<double> expi_turns(uint64_t t) {
    const uint32_t q = (uint32_t)(((t + (1ull << 61)) >> 62) & 3u);
    const int64_t r = (int64_t)(t - ((uint64_t)q << 62));
    const double x = (double)r * 3.4061215800865545e-19;  // 2 pi / 2^64
    const double x2 = x * x;
    // 1/(2k+1)! and 1/(2k)! by Horner from the highest term
    double ps = 1.0 / 355687428096000.0;            // 1/17!
    ps = ps * x2 - 1.0 / 1307674368000.0;           // 1/15!
    ps = ps * x2 + 1.0 / 6227020800.0;              // 1/13!
    ps = ps * x2 - 1.0 / 39916800.0;                // 1/11!
    ps = ps * x2 + 1.0 / 362880.0;                  // 1/9!
    ps = ps * x2 - 1.0 / 5040.0;
    ps = ps * x2 + 1.0 / 120.0;
    ps = ps * x2 - 1.0 / 6.0;
    ps = ps * x2 + 1.0;
    double pc = 1.0 / 6402373705728000.0;           // 1/18!
    pc = pc * x2 - 1.0 / 20922789888000.0;          // 1/16!
    pc = pc * x2 + 1.0 / 87178291200.0;             // 1/14!
    pc = pc * x2 - 1.0 / 479001600.0;               // 1/12!
    pc = pc * x2 + 1.0 / 3628800.0;                 // 1/10!
    pc = pc * x2 - 1.0 / 40320.0;
    pc = pc * x2 + 1.0 / 720.0;
    pc = pc * x2 - 1.0 / 24.0;
    pc = pc * x2 + 0.5;
    pc = 1.0 - pc * x2;
    const double sn = x * ps;
    const bool odd = (q & 1u) != 0;
    cplx<double> e = {odd ? sn : pc, odd ? pc : sn};
    return cneg_parts(e, ((q + 1u) >> 1) & 1u, q >> 1);
}

// Phase accumulator type: 32-bit turns at complex64, 64-bit at complex128.
template <typename R>
struct Turns;
template <>
struct Turns<float> {
    using T = uint32_t;
};
template <>
struct Turns<double> {
    using T = uint64_t;
};

template <int N>
using IC = std::integral_constant<int, N>;

// Compile-time loop: f(IC<0>{}), .., f(IC<N-1>{}) -- every register index
// stays a constant, so the tile never leaves registers.
template <typename F, int... Is>
__device__ __forceinline__ void sfor_impl(F &&f, std::integer_sequence<int, Is...>) {
    (f(IC<Is>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void sfor(F &&f) {
    sfor_impl(f, std::make_integer_sequence<int, N>{});
}

// Call f(IC<i>) for a runtime register bit i < RB.
template <int RB, typename F>
__device__ __forceinline__ void with_reg(uint32_t i, F &&f) {
    switch (i) {
        case 0: if constexpr (RB > 0) f(IC<0>{}); break;
        case 1: if constexpr (RB > 1) f(IC<1>{}); break;
        case 2: if constexpr (RB > 2) f(IC<2>{}); break;
        case 3: if constexpr (RB > 3) f(IC<3>{}); break;
        case 4: if constexpr (RB > 4) f(IC<4>{}); break;
        case 5: if constexpr (RB > 5) f(IC<5>{}); break;
        default: break;
    }
}

// Frame-conjugated 2x2 / 4x4 entry: G[(r^x) * k + (c^x)] (-1)^{z.r + z.c}
template <typename R>
__device__ __forceinline__ cplx<R> conj_entry(kptr<cplx<R>> G, uint32_t k, uint32_t r, uint32_t c,
                                              uint32_t xl, uint32_t zl) {
    const cplx<R> v = G[(r ^ xl) * k + (c ^ xl)];
    return cneg_if(v, (__builtin_popcount(zl & r) + __builtin_popcount(zl & c)) & 1u);
}

// ---------------------------------------------------------------- DENSE1 --
// 2x2 on the target qubit; with nq == 2 the gate is block-diagonal in the
// other (control) qubit and the control's value selects the block.
template <bool REAL, typename R>
__device__ __forceinline__ cplx<R> mmul(cplx<R> m, cplx<R> x) {
    if constexpr (REAL) return rmul(m, x);
    else return cmul(m, x);
}
template <bool REAL, typename R>
__device__ __forceinline__ cplx<R> mmac(cplx<R> a, cplx<R> m, cplx<R> x) {
    if constexpr (REAL) return rmac(a, m, x);
    else return cmac(a, m, x);
}

// Target on register bit I: one 2x2 M for every pair (M wave-uniform, or
// per lane when a lane qubit controls it).
template <typename R, int RB, bool REAL, int I>
__device__ __forceinline__ void d1_reg(cplx<R> (&v)[1 << RB], const cplx<R> (&M)[4]) {
    sfor<(1 << RB)>([&](auto Jc) __attribute__((always_inline)) {
        constexpr int j = decltype(Jc)::value;
        if constexpr (!(j & (1 << I))) {
            const cplx<R> x0 = v[j], x1 = v[j | (1 << I)];
            v[j] = mmac<REAL>(mmul<REAL>(M[0], x0), M[1], x1);
            v[j | (1 << I)] = mmac<REAL>(mmul<REAL>(M[2], x0), M[3], x1);
        }
    });
}

// Target on register bit I, control on register bit cpos: the block of each
// pair is chosen by a wave-uniform bit of its register index.
template <typename R, int RB, bool REAL, int I>
__device__ __forceinline__ void d1_reg_ctrl(cplx<R> (&v)[1 << RB], const cplx<R> (&B)[2][4], uint32_t cpos) {
    sfor<(1 << RB)>([&](auto Jc) __attribute__((always_inline)) {
        constexpr int j = decltype(Jc)::value;
        if constexpr (!(j & (1 << I))) {
            const bool cb = (((uint32_t)j >> cpos) & 1u) != 0;
            const cplx<R> x0 = v[j], x1 = v[j | (1 << I)];
            const cplx<R> m0 = csel(cb, B[1][0], B[0][0]), m1 = csel(cb, B[1][1], B[0][1]);
            const cplx<R> m2 = csel(cb, B[1][2], B[0][2]), m3 = csel(cb, B[1][3], B[0][3]);
            v[j] = mmac<REAL>(mmul<REAL>(m0, x0), m1, x1);
            v[j | (1 << I)] = mmac<REAL>(mmul<REAL>(m2, x0), m3, x1);
        }
        shuffle_fence<j>();
    });
}

// Target on a lane bit: own row b, partner (lane ^ mask) column 1 - b; with
// a register control the row pair (a, c) comes from block 0 or 1 per index.
template <typename R, int RB, bool REAL, bool CREG>
__device__ __forceinline__ void d1_lane(cplx<R> (&v)[1 << RB], uint32_t mask, cplx<R> a0, cplx<R> c0,
                                        cplx<R> a1, cplx<R> c1, uint32_t cpos) {
    sfor<(1 << RB)>([&](auto Jc) __attribute__((always_inline)) {
        constexpr int j = decltype(Jc)::value;
        const cplx<R> p = shfl_xor_c(v[j], mask);
        cplx<R> a = a0, c = c0;
        if constexpr (CREG) {
            const bool cb = (((uint32_t)j >> cpos) & 1u) != 0;
            a = csel(cb, a1, a0);
            c = csel(cb, c1, c0);
        }
        v[j] = mmac<REAL>(mmul<REAL>(a, v[j]), c, p);
        shuffle_fence<j>();
    });
}

template <typename R, int RB, bool REAL>
__device__ __forceinline__ void dense1_apply(cplx<R> (&v)[1 << RB], const cplx<R> (&B)[2][4], uint32_t crole,
                                             uint32_t cpos, uint32_t base, uint32_t trole, uint32_t tpos,
                                             uint32_t L) {
    const bool creg = crole == ROLE_REG;
    if (trole == ROLE_REG) {
        if (creg) {
            with_reg<RB>(tpos, [&](auto Ic) __attribute__((always_inline)) {
                d1_reg_ctrl<R, RB, REAL, decltype(Ic)::value>(v, B, cpos);
            });
        } else {
            // no control, or a control fixed for the tile / the lane
            uint32_t cb = 0;
            if (crole == ROLE_FIXED) cb = (base >> cpos) & 1u;
            else if (crole == ROLE_LANE) cb = (L >> cpos) & 1u;
            cplx<R> M[4];
#pragma unroll
            for (int e = 0; e < 4; e++) M[e] = csel(cb != 0, B[1][e], B[0][e]);
            with_reg<RB>(tpos, [&](auto Ic) __attribute__((always_inline)) {
                d1_reg<R, RB, REAL, decltype(Ic)::value>(v, M);
            });
        }
    } else {
        const uint32_t b = (L >> tpos) & 1u;
        cplx<R> a0 = csel(b != 0, B[0][3], B[0][0]), c0 = csel(b != 0, B[0][2], B[0][1]);
        const cplx<R> a1 = csel(b != 0, B[1][3], B[1][0]), c1 = csel(b != 0, B[1][2], B[1][1]);
        if (creg) {
            d1_lane<R, RB, REAL, true>(v, 1u << tpos, a0, c0, a1, c1, cpos);
        } else {
            uint32_t cb = 0;
            if (crole == ROLE_FIXED) cb = (base >> cpos) & 1u;
            else if (crole == ROLE_LANE) cb = (L >> cpos) & 1u;
            a0 = csel(cb != 0, a1, a0);
            c0 = csel(cb != 0, c1, c0);
            d1_lane<R, RB, REAL, false>(v, 1u << tpos, a0, c0, a1, c1, 0);
        }
    }
}

template <typename R, int RB>
__device__ __forceinline__ void op_dense1(cplx<R> (&v)[1 << RB], const OpDesc &o, kptr<cplx<R>> G,
                                          uint32_t xl, uint32_t zl, uint32_t L, uint32_t base) {
    const uint32_t tq = o.nq == 2 ? o.tq : 0u, cq = 1u - tq;
    const uint32_t k = 1u << o.nq;
    cplx<R> B[2][4];
#pragma unroll
    for (uint32_t cb = 0; cb < 2; cb++)
#pragma unroll
        for (uint32_t rr = 0; rr < 2; rr++)
#pragma unroll
            for (uint32_t cc = 0; cc < 2; cc++) {
                uint32_t r = rr << tq, c = cc << tq;
                if (o.nq == 2) {
                    r |= cb << cq;
                    c |= cb << cq;
                }
                B[cb][rr * 2 + cc] = conj_entry(G, k, r, c, xl, zl);
            }
    // control role: none (one-qubit gate: both blocks are the gate), a
    // register, lane or tile-fixed qubit
    const uint32_t crole = o.nq == 2 ? (cq ? o.role[1] : o.role[0]) : 0xFFu;
    const uint32_t cpos = cq ? o.pos[1] : o.pos[0];
    const uint32_t trole = tq ? o.role[1] : o.role[0];
    const uint32_t tpos = tq ? o.pos[1] : o.pos[0];
    if (o.real) dense1_apply<R, RB, true>(v, B, crole, cpos, base, trole, tpos, L);
    else dense1_apply<R, RB, false>(v, B, crole, cpos, base, trole, tpos, L);
}

// ---------------------------------------------------------------- DENSE2 --
// 4x4 on register bits A < B (normalised qubit order).
template <typename R, int RB, int A, int Bb>
__device__ __forceinline__ void dense2_rr(cplx<R> (&v)[1 << RB], const cplx<R> (&M)[16]) {
    sfor<(1 << RB)>([&](auto Jc) __attribute__((always_inline)) {
        constexpr int j = decltype(Jc)::value;
        if constexpr (!(j & ((1 << A) | (1 << Bb)))) {
            constexpr int i0 = j, i1 = j | (1 << A), i2 = j | (1 << Bb);
            constexpr int i3 = j | (1 << A) | (1 << Bb);
            const cplx<R> x0 = v[i0], x1 = v[i1], x2 = v[i2], x3 = v[i3];
            v[i0] = cmac(cmac(cmac(cmul(M[0], x0), M[1], x1), M[2], x2), M[3], x3);
            v[i1] = cmac(cmac(cmac(cmul(M[4], x0), M[5], x1), M[6], x2), M[7], x3);
            v[i2] = cmac(cmac(cmac(cmul(M[8], x0), M[9], x1), M[10], x2), M[11], x3);
            v[i3] = cmac(cmac(cmac(cmul(M[12], x0), M[13], x1), M[14], x2), M[15], x3);
        }
        shuffle_fence<j>();
    });
}

template <typename R, int RB, int A>
__device__ __forceinline__ void dense2_rr_b(cplx<R> (&v)[1 << RB], const cplx<R> (&M)[16], uint32_t b) {
    switch (b) {
        case 1: if constexpr (RB > 1 && A < 1) dense2_rr<R, RB, A, 1>(v, M); break;
        case 2: if constexpr (RB > 2 && A < 2) dense2_rr<R, RB, A, 2>(v, M); break;
        case 3: if constexpr (RB > 3 && A < 3) dense2_rr<R, RB, A, 3>(v, M); break;
        case 4: if constexpr (RB > 4 && A < 4) dense2_rr<R, RB, A, 4>(v, M); break;
        case 5: if constexpr (RB > 5 && A < 5) dense2_rr<R, RB, A, 5>(v, M); break;
        default: break;
    }
}

template <typename R, int RB>
__device__ __forceinline__ void dense2_rr_dispatch(cplx<R> (&v)[1 << RB], const cplx<R> (&M)[16],
                                                   uint32_t a, uint32_t b) {
    switch (a) {
        case 0: dense2_rr_b<R, RB, 0>(v, M, b); break;
        case 1: dense2_rr_b<R, RB, 1>(v, M, b); break;
        case 2: dense2_rr_b<R, RB, 2>(v, M, b); break;
        case 3: dense2_rr_b<R, RB, 3>(v, M, b); break;
        case 4: dense2_rr_b<R, RB, 4>(v, M, b); break;
        default: break;
    }
}

template <typename R, int RB>
__device__ __forceinline__ void op_dense2(cplx<R> (&v)[1 << RB], const OpDesc &o, kptr<cplx<R>> G,
                                          uint32_t xl, uint32_t zl, uint32_t L) {
    constexpr int NJ = 1 << RB;
    // M[r][c] in the gate's qubit order, frame-conjugated
    const bool r0 = o.role[0] == ROLE_REG, r1 = o.role[1] == ROLE_REG;
    // normalised order: first qubit = the register one (or lower register bit)
    bool swapq = false;
    if (r0 && r1) swapq = o.pos[0] > o.pos[1];
    else if (!r0 && r1) swapq = true;
    cplx<R> M[16];
#pragma unroll
    for (uint32_t r = 0; r < 4; r++)
#pragma unroll
        for (uint32_t c = 0; c < 4; c++) {
            const uint32_t rs = swapq ? ((r >> 1) | ((r & 1u) << 1)) : r;
            const uint32_t cs = swapq ? ((c >> 1) | ((c & 1u) << 1)) : c;
            M[r * 4 + c] = conj_entry(G, 4, rs, cs, xl, zl);
        }
    const uint32_t p0 = swapq ? o.pos[1] : o.pos[0];
    const uint32_t p1 = swapq ? o.pos[0] : o.pos[1];
    if (r0 && r1) {
        dense2_rr_dispatch<R, RB>(v, M, p0, p1);
    } else if (r0 || r1) {
        // qubit 0 (normalised) in register bit p0, qubit 1 on lane bit p1:
        // own rows 2b, 2b+1; columns own (2b, 2b+1), partner (2-2b, 3-2b)
        const uint32_t b = (L >> p1) & 1u, mask = 1u << p1;
        cplx<R> k0[4], k1[4];
#pragma unroll
        for (uint32_t cc = 0; cc < 4; cc++) {
            const cplx<R> e0_b0 = M[0 * 4 + (cc == 0 ? 0 : cc == 1 ? 1 : cc == 2 ? 2 : 3)];
            const cplx<R> e0_b1 = M[2 * 4 + (cc == 0 ? 2 : cc == 1 ? 3 : cc == 2 ? 0 : 1)];
            const cplx<R> e1_b0 = M[1 * 4 + (cc == 0 ? 0 : cc == 1 ? 1 : cc == 2 ? 2 : 3)];
            const cplx<R> e1_b1 = M[3 * 4 + (cc == 0 ? 2 : cc == 1 ? 3 : cc == 2 ? 0 : 1)];
            k0[cc] = csel(b != 0, e0_b1, e0_b0);
            k1[cc] = csel(b != 0, e1_b1, e1_b0);
        }
        with_reg<RB>(p0, [&](auto Ia) __attribute__((always_inline)) {
            constexpr int A = decltype(Ia)::value;
            sfor<NJ>([&](auto Jc) __attribute__((always_inline)) {
                constexpr int j = decltype(Jc)::value;
                if constexpr (j & (1 << A)) return;
                const cplx<R> a0 = v[j], a1 = v[j | (1 << A)];
                const cplx<R> q0 = shfl_xor_c(a0, mask), q1 = shfl_xor_c(a1, mask);
                cplx<R> n0, n1;
                if (o.real) {
                    n0 = rmac(rmac(rmac(rmul(k0[0], a0), k0[1], a1), k0[2], q0), k0[3], q1);
                    n1 = rmac(rmac(rmac(rmul(k1[0], a0), k1[1], a1), k1[2], q0), k1[3], q1);
                } else {
                    n0 = cmac(cmac(cmac(cmul(k0[0], a0), k0[1], a1), k0[2], q0), k0[3], q1);
                    n1 = cmac(cmac(cmac(cmul(k1[0], a0), k1[1], a1), k1[2], q0), k1[3], q1);
                }
                v[j] = n0;
                v[j | (1 << A)] = n1;
                shuffle_fence<j>();
            });
        });
    } else {
        // both on lanes: own index r = b0 + 2 b1, partners r^1, r^2, r^3
        const uint32_t b0 = (L >> p0) & 1u, b1 = (L >> p1) & 1u;
        const uint32_t m0 = 1u << p0, m1 = 1u << p1;
        const uint32_t r = b0 | (b1 << 1);
        cplx<R> k[4];
#pragma unroll
        for (uint32_t d = 0; d < 4; d++) {
            const cplx<R> e0 = M[0 * 4 + (0 ^ d)], e1 = M[1 * 4 + (1 ^ d)];
            const cplx<R> e2 = M[2 * 4 + (2 ^ d)], e3 = M[3 * 4 + (3 ^ d)];
            k[d] = csel(r == 3, e3, csel(r == 2, e2, csel(r == 1, e1, e0)));
        }
        sfor<NJ>([&](auto Jc) __attribute__((always_inline)) {
            constexpr int j = decltype(Jc)::value;
            const cplx<R> q1 = shfl_xor_c(v[j], m0);
            const cplx<R> q2 = shfl_xor_c(v[j], m1);
            const cplx<R> q3 = shfl_xor_c(v[j], m0 | m1);
            v[j] = cmac(cmac(cmac(cmul(k[0], v[j]), k[1], q1), k[2], q2), k[3], q3);
            shuffle_fence<j>();
        });
    }
}

// ------------------------------------------------------------ DIAG gates --
// One diagonal gate, gate-by-gate path: d'(r) = d(r ^ x).
template <typename R, int RB>
__device__ __forceinline__ void op_diag_one(cplx<R> (&v)[1 << RB], const DiagGate &dg, kptr<cplx<R>> D,
                                            uint32_t fx, uint32_t L, uint32_t base) {
    constexpr int NJ = 1 << RB;
    uint32_t xl = (fx >> dg.phys[0]) & 1u;
    if (dg.nq == 2) xl |= ((fx >> dg.phys[1]) & 1u) << 1;
    const uint32_t nd = 1u << dg.nq;
    cplx<R> d[4];
#pragma unroll
    for (uint32_t r = 0; r < 4; r++) d[r] = D[(r & (nd - 1u)) ^ xl];
    uint32_t rb = 0;  // bits that do not depend on j
    uint32_t regpos[2] = {0, 0};
    bool isreg[2] = {false, false};
#pragma unroll
    for (uint32_t q = 0; q < 2; q++) {
        if (q >= dg.nq) break;
        const uint32_t role = q ? dg.role[1] : dg.role[0];
        const uint32_t pos = q ? dg.pos[1] : dg.pos[0];
        if (role == ROLE_LANE) rb |= ((L >> pos) & 1u) << q;
        else if (role == ROLE_FIXED) rb |= ((base >> pos) & 1u) << q;
        else {
            isreg[q] = true;
            regpos[q] = pos;
        }
    }
    sfor<NJ>([&](auto Jc) __attribute__((always_inline)) {
        constexpr int j = decltype(Jc)::value;
        uint32_t r = rb;
        if (isreg[0]) r |= ((uint32_t)j >> regpos[0]) & 1u;
        if (isreg[1]) r |= (((uint32_t)j >> regpos[1]) & 1u) << 1;
        const cplx<R> lo = csel((r & 1u) != 0, d[1], d[0]);
        const cplx<R> hi = csel((r & 1u) != 0, d[3], d[2]);
        v[j] = cmul(csel((r & 2u) != 0, hi, lo), v[j]);
    });
}

// The run's phase factors applied with one multiply per amplitude (plus one
// per register-dependent coefficient): e^{2 pi i (C + sum_i lam_i x_i)}.
template <typename R, int RB>
__device__ __forceinline__ void apply_run_phase(cplx<R> (&v)[1 << RB], typename Turns<R>::T C,
                                                const typename Turns<R>::T (&lam)[RB], uint32_t lm) {
    constexpr int NJ = 1 << RB;
    constexpr int LO = RB < 3 ? RB : 3;
    constexpr int HI = RB - LO;
    if (__builtin_popcount(lm) == 1) {
        // one register-dependent factor: e^{2 pi i C} on the registers with
        // the bit clear, e^{2 pi i (C + lam_i)} on the others
        with_reg<RB>((uint32_t)__builtin_ctz(lm), [&](auto Ic) __attribute__((always_inline)) {
            constexpr int I = decltype(Ic)::value;
            const cplx<R> w0 = expi_turns(C);
            const cplx<R> w1 = cmul(w0, expi_turns(lam[I]));
            sfor<NJ>([&](auto Jc) __attribute__((always_inline)) {
                constexpr int j = decltype(Jc)::value;
                v[j] = cmul(((j >> I) & 1) ? w1 : w0, v[j]);
            });
        });
    } else if (__builtin_popcount(lm) <= 2) {
        // few register-dependent factors: e^{2 pi i C}, then e^{2 pi i lam_i}
        // on the registers with bit i set
        const cplx<R> w0 = expi_turns(C);
        sfor<NJ>([&](auto Jc) __attribute__((always_inline)) {
            constexpr int j = decltype(Jc)::value;
            v[j] = cmul(w0, v[j]);
        });
        sfor<RB>([&](auto Ic) __attribute__((always_inline)) {
            constexpr int i = decltype(Ic)::value;
            if ((lm >> i) & 1u) {
                const cplx<R> e = expi_turns(lam[i]);
                sfor<NJ>([&](auto Jc) __attribute__((always_inline)) {
                    constexpr int j = decltype(Jc)::value;
                    if constexpr (((j >> i) & 1) != 0) v[j] = cmul(e, v[j]);
                });
            }
        });
    } else {
        // subset products over the low and high register bits
        cplx<R> wlo[1 << LO], whi[1 << HI];
        wlo[0] = expi_turns(C);
        sfor<LO>([&](auto Ic) __attribute__((always_inline)) {
            constexpr int i = decltype(Ic)::value;
            const cplx<R> e = expi_turns(lam[i]);
            sfor<(1 << i)>([&](auto Sc) __attribute__((always_inline)) {
                constexpr int s2 = decltype(Sc)::value;
                wlo[s2 | (1 << i)] = cmul(wlo[s2], e);
            });
        });
        whi[0] = cplx<R>{R(1), R(0)};
        sfor<HI>([&](auto Ic) __attribute__((always_inline)) {
            constexpr int i = decltype(Ic)::value;
            const cplx<R> e = expi_turns(lam[LO + i]);
            sfor<(1 << i)>([&](auto Sc) __attribute__((always_inline)) {
                constexpr int s2 = decltype(Sc)::value;
                whi[s2 | (1 << i)] = cmul(whi[s2], e);
            });
        });
        sfor<NJ>([&](auto Jc) __attribute__((always_inline)) {
            constexpr int j = decltype(Jc)::value;
            const cplx<R> w = HI ? cmul(wlo[j & ((1 << LO) - 1)], whi[j >> LO]) : wlo[j & ((1 << LO) - 1)];
            v[j] = cmul(w, v[j]);
        });
    }
}

// The X part of the frame along a phase run with up to three noise events
// inside it: gates [0, k0) see f0, [k0, k1) f1, [k1, k2) f2, the rest f3
// (only the X part matters for diagonal gates).
struct RunFrames {
    uint32_t k0, k1, k2;
    uint32_t f0, f1, f2, f3;
    __device__ __forceinline__ uint32_t at(uint32_t k) const {
        return k < k0 ? f0 : (k < k1 ? f1 : (k < k2 ? f2 : f3));
    }
};

// A phase run split by noise events: the same phase polynomial as
// op_diag_run, with each term evaluated in its own gate's frame and the
// register-bit frame folded in per term; the gates on register qubits only
// are applied one by one by the caller.
template <typename R, int RB>
__device__ __forceinline__ void op_diag_run_split(cplx<R> (&v)[1 << RB], const OpDesc &o, kptr<DiagTerm> tm,
                                                  const RunFrames &rf, uint32_t L, uint32_t base,
                                                  const uint32_t (&rq)[RB]) {
    using A = typename Turns<R>::T;
    A C = 0;
    A lam[RB];
#pragma unroll
    for (int i = 0; i < RB; i++) lam[i] = 0;
    kptr<DiagTerm> p = tm;
    for (uint32_t k = 0; k < o.n_fix; k++) {
        const TermU<A> t = load_term<A>(p + k);
        const uint32_t yfix = base ^ rf.at(t.k);
        const uint32_t y0 = (yfix >> t.phys0) & 1u;
        const uint32_t y1 = t.nq == 2 ? (yfix >> t.phys1) & 1u : 0u;
        const A lo = y0 ? t.th[1] : t.th[0], hi = y0 ? t.th[3] : t.th[2];
        C += y1 ? hi : lo;
    }
    p += o.n_fix;
    sfor<RB>([&](auto Ic) __attribute__((always_inline)) {
        constexpr int i = decltype(Ic)::value;
        const uint32_t cnt = o.n_fixreg[i];
        for (uint32_t k = 0; k < cnt; k++) {
            const TermU<A> t = load_term<A>(p + k);
            const uint32_t f = rf.at(t.k);
            const uint32_t y = ((base ^ f) >> t.phys0) & 1u;
            const A a0 = y ? t.th[1] : t.th[0], a1 = y ? t.th[3] : t.th[2];
            // register value x_i ^ f_i: a0 + (a1 - a0) (x_i ^ f_i)
            const bool fi = ((f >> rq[i]) & 1u) != 0;
            C += fi ? a1 : a0;
            lam[i] += fi ? (A)(a0 - a1) : (A)(a1 - a0);
        }
        p += cnt;
    });
    for (uint32_t k = 0; k < o.n_lane; k++) {
        const TermU<A> t = load_term<A>(p + k);
        const uint32_t f = rf.at(t.k);
        const uint32_t ylane = L ^ f, yfix = base ^ f;
        const uint32_t y0 = (ylane >> t.phys0) & 1u;
        if (t.nq == 1) {
            C += y0 ? t.th[1] : t.th[0];
        } else {
            const uint32_t y1 = t.role1 == ROLE_LANE ? (ylane >> t.phys1) & 1u : (yfix >> t.phys1) & 1u;
            const A lo = y0 ? t.th[1] : t.th[0], hi = y0 ? t.th[3] : t.th[2];
            C += y1 ? hi : lo;
        }
    }
    p += o.n_lane;
    sfor<RB>([&](auto Ic) __attribute__((always_inline)) {
        constexpr int i = decltype(Ic)::value;
        const uint32_t cnt = o.n_lanereg[i];
        for (uint32_t k = 0; k < cnt; k++) {
            const TermU<A> t = load_term<A>(p + k);
            const uint32_t f = rf.at(t.k);
            const uint32_t y = ((L ^ f) >> t.phys0) & 1u;
            const A a0 = y ? t.th[1] : t.th[0], a1 = y ? t.th[3] : t.th[2];
            const bool fi = ((f >> rq[i]) & 1u) != 0;
            C += fi ? a1 : a0;
            lam[i] += fi ? (A)(a0 - a1) : (A)(a1 - a0);
        }
        p += cnt;
    });
    apply_run_phase<R, RB>(v, C, lam, o.lam_mask);
}

// A run of diagonal gates as one phase polynomial (all its gates commute).
// With y = index ^ frame-x, the run's phase (in turns) is
//   C(lane, fixed bits) + sum_i lam_i(lane, fixed bits) y_reg_i + P(y_reg).
// Gates on register qubits only form the table T = e^{2 pi i P} (host side);
// the other terms arrive grouped: fixed-only and fixed+register terms give
// wave-uniform contributions, lane and lane+register terms per-lane ones.
template <typename R, int RB>
__device__ __forceinline__ void op_diag_run(cplx<R> (&v)[1 << RB], const OpDesc &o, kptr<cplx<R>> T,
                                            kptr<DiagTerm> tm, uint32_t fx, uint32_t L, uint32_t base,
                                            const uint32_t (&rq)[RB], uint32_t nr) {
    using A = typename Turns<R>::T;
    constexpr int NJ = 1 << RB;
    const uint32_t yfix = base ^ fx;  // frame-adjusted fixed bits (uniform)
    const uint32_t ylane = L ^ fx;    // frame-adjusted lane bits (lane qubits are physical 0..5)
    // wave-uniform part
    A Cu = 0;
    A lamu[RB];
#pragma unroll
    for (int i = 0; i < RB; i++) lamu[i] = 0;
    kptr<DiagTerm> p = tm;
    for (uint32_t k = 0; k < o.n_fix; k++) {
        const TermU<A> t = load_term<A>(p + k);
        const uint32_t y0 = (yfix >> t.phys0) & 1u;
        const uint32_t y1 = t.nq == 2 ? (yfix >> t.phys1) & 1u : 0u;
        const A t0 = t.th[0], t1 = t.th[1], t2 = t.th[2], t3 = t.th[3];
        const A lo = y0 ? t1 : t0, hi = y0 ? t3 : t2;
        Cu += y1 ? hi : lo;
    }
    p += o.n_fix;
    sfor<RB>([&](auto Ic) __attribute__((always_inline)) {
        constexpr int i = decltype(Ic)::value;
        const uint32_t cnt = o.n_fixreg[i];
        A cs = 0, ls = 0;
        for (uint32_t k = 0; k < cnt; k++) {
            const TermU<A> t = load_term<A>(p + k);
            const uint32_t y = (yfix >> t.phys0) & 1u;
            const A t0 = t.th[0], t1 = t.th[1], t2 = t.th[2], t3 = t.th[3];
            const A a0 = y ? t1 : t0, a1 = y ? t3 : t2;
            cs += a0;
            ls += a1 - a0;
        }
        Cu += cs;
        lamu[i] += ls;
        p += cnt;
    });
    // per-lane part
    A C = Cu;
    A lam[RB];
#pragma unroll
    for (int i = 0; i < RB; i++) lam[i] = lamu[i];
#pragma unroll 2
    for (uint32_t k = 0; k < o.n_lane; k++) {
        const TermU<A> t = load_term<A>(p + k);
        const uint32_t y0 = (ylane >> t.phys0) & 1u;
        const A t0 = t.th[0], t1 = t.th[1], t2 = t.th[2], t3 = t.th[3];
        if (t.nq == 1) {
            C += y0 ? t1 : t0;
        } else {
            const uint32_t y1 = t.role1 == ROLE_LANE ? (ylane >> t.phys1) & 1u : (yfix >> t.phys1) & 1u;
            const A lo = y0 ? t1 : t0, hi = y0 ? t3 : t2;
            C += y1 ? hi : lo;
        }
    }
    p += o.n_lane;
    sfor<RB>([&](auto Ic) __attribute__((always_inline)) {
        constexpr int i = decltype(Ic)::value;
        const uint32_t cnt = o.n_lanereg[i];
#pragma unroll 2
        for (uint32_t k = 0; k < cnt; k++) {
            const TermU<A> t = load_term<A>(p + k);
            const uint32_t y = (ylane >> t.phys0) & 1u;
            const A t0 = t.th[0], t1 = t.th[1], t2 = t.th[2], t3 = t.th[3];
            const A a0 = y ? t1 : t0;
            const A a1 = y ? t3 : t2;
            C += a0;
            lam[i] += a1 - a0;
        }
        p += cnt;
    });
    // register bits: y_i = x_i ^ f_i, so lam_i y_i = f_i lam_i + (-1)^{f_i} lam_i x_i
    uint32_t fr = 0;
    sfor<RB>([&](auto Ic) __attribute__((always_inline)) {
        constexpr int i = decltype(Ic)::value;
        if ((uint32_t)i < nr) {
            const uint32_t f = (fx >> rq[i]) & 1u;
            fr |= f << i;
            if (f) {
                C += lam[i];
                lam[i] = (A)0 - lam[i];
            }
        }
    });
    apply_run_phase<R, RB>(v, C, lam, o.lam_mask);
    if (o.has_t) {
        // register-only gates: one wave-uniform factor per register index
        const uint32_t msk = (1u << nr) - 1u;
        sfor<NJ>([&](auto Jc) __attribute__((always_inline)) {
            constexpr int j = decltype(Jc)::value;
            const uint32_t t = ((uint32_t)j ^ fr) & msk;
            if (t >= 32u || ((o.tmask >> t) & 1u)) v[j] = cmul(T[t], v[j]);
        });
    }
}

// ------------------------------------------------------------------ kernel --
// D2: the pass contains 4x4 ops (a separate instantiation keeps the
// register budget of the common passes small).
// Waves per SIMD the register allocator is held to: three for the
// complex64 tiles of up to 32 amplitudes per lane (at most 168 registers),
// no bound for the larger tiles, whose registers hold the tile itself.
template <typename R, int RB>
struct PassWaves {
    static constexpr int value = (sizeof(R) == 4 && RB <= 5) ? 3 : 1;
};

// Sampling partials of a full tile (64 lanes, RB registers) in the final
// layout: |amplitude|^2 in FP64, summed over the in-block positions that
// vary inside the tile (registers by pairs, lanes by shuffles), leaving one
// mass per pattern of the block-index positions that vary inside it.
// Pattern bits: the block-index lane positions in increasing order, then
// the block-index register bits in register order.  Written to
// part[(state * tiles + tile) << kv | pattern], each lane holding a pattern
// of its own for every remaining register index.
template <typename R, int RB>
__device__ __forceinline__ void tile_partials(const cplx<R> (&v)[1 << RB], const PassArgs<R> &a, uint32_t traj,
                                              uint32_t tile, uint32_t nfree, uint32_t L) {
    constexpr int NJ = 1 << RB;
    const uint32_t fold_l = a.psum & 0xFFu, fold_r = (a.psum >> 8) & 0xFFu, kv = (a.psum >> 16) & 0xFFu;
    double p[NJ];
    sfor<NJ>([&](auto Jc) __attribute__((always_inline)) {
        constexpr int j = decltype(Jc)::value;
        p[j] = (double)v[j].re * (double)v[j].re + (double)v[j].im * (double)v[j].im;
    });
    sfor<RB>([&](auto Ic) __attribute__((always_inline)) {
        constexpr int i = decltype(Ic)::value;
        if ((fold_r >> i) & 1u) {
            sfor<NJ>([&](auto Jc) __attribute__((always_inline)) {
                constexpr int j = decltype(Jc)::value;
                if constexpr (!(j & (1 << i))) p[j] += p[j | (1 << i)];
            });
        }
    });
    for (uint32_t b = 0; b < kLaneBits; b++) {
        if (!((fold_l >> b) & 1u)) continue;
        sfor<NJ>([&](auto Jc) __attribute__((always_inline)) {
            constexpr int j = decltype(Jc)::value;
            if (((uint32_t)j & fold_r) == 0) p[j] += __shfl_xor(p[j], (int)(1u << b));
        });
    }
    if (L & fold_l) return;
    // lane pattern: the lane's block-index bits, compressed
    uint32_t lp = 0, nlc = 0;
    for (uint32_t b = 0; b < kLaneBits; b++)
        if (!((fold_l >> b) & 1u)) lp |= ((L >> b) & 1u) << nlc++;
    double *out = a.part + (((uint64_t)traj << nfree | tile) << kv);
    sfor<NJ>([&](auto Jc) __attribute__((always_inline)) {
        constexpr int j = decltype(Jc)::value;
        if (((uint32_t)j & fold_r) == 0) {
            uint32_t rp = 0, nrc = 0;
            sfor<RB>([&](auto Ic) __attribute__((always_inline)) {
                constexpr int i = decltype(Ic)::value;
                if (!((fold_r >> i) & 1u)) rp |= (uint32_t)((j >> i) & 1) << nrc++;
            });
            out[lp | (rp << nlc)] = p[j];
        }
    });
}

template <typename R, int RB, bool D2>
__global__ __launch_bounds__(64, (PassWaves<R, RB>::value)) void pass_kernel(PassLaunch<R> pl) {
    constexpr int NJ = 1 << RB;
    const uint32_t nwg = gridDim.x, bid = blockIdx.x;
    const uint32_t wall = (bid & 7u) * (nwg >> 3) + (bid >> 3);
    if (wall >= pl.total) return;
    PassArgs<R> a;
    uint32_t w = wall;
    if (pl.nseg == 0) {
        a = pl.one;
    } else {
        // the last segment starting at or before this workgroup
        const kptr<PassArgs<R>> segs = kconst(pl.segs);
        uint32_t lo = 0, hi = pl.nseg;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (segs[mid].wg_begin <= wall) lo = mid;
            else hi = mid;
        }
        a = kload(segs + lo);
        w = wall - a.wg_begin;
    }
    if (w >= a.work) return;
    const uint32_t traj = w % a.count, tile = w / a.count;
    const uint32_t L = threadIdx.x;
    const kptr<PassDesc> pd = kconst(a.pass);
    const kptr<OpDesc> ops = kconst(a.ops);
    const kptr<cplx<R>> mats = kconst(a.mats);
    const kptr<uint32_t> ev_pos = kconst(a.meta.ev_pos), ev_dx = kconst(a.meta.ev_dx),
                         ev_dz = kconst(a.meta.ev_dz);
    static_assert(offsetof(PassDesc, nl) == 8 && offsetof(PassDesc, rq) == 12 && offsetof(PassDesc, fbits) == 20,
                  "pass descriptor layout");
    const kptr<uint32_t> pw = (kptr<uint32_t>)pd;
    const uint32_t op_begin = uni(pw[0]), op_count = uni(pw[1]), pw2 = uni(pw[2]);
    const uint32_t rq03 = uni(pw[3]), rq47 = uni(pw[4]);
    const uint32_t nl = pw2 & 0xFFu, nr = (pw2 >> 8) & 0xFFu, nfree = (pw2 >> 16) & 0xFFu;

    // tile loads go out first; the noise metadata is fetched behind them
    const uint32_t src_s = kconst(a.src_slot)[traj];
    const uint32_t dst_s = kconst(a.dst_slot)[traj];
    uint32_t base = 0;
    for (uint32_t i = 0; i < nfree; i++) base |= ((tile >> i) & 1u) << ((uni(pw[5 + (i >> 2)]) >> (8 * (i & 3u))) & 0xFFu);
    uint32_t rq[RB];
#pragma unroll
    for (int i = 0; i < RB; i++) rq[i] = (uint32_t)i < nr ? (((i < 4 ? rq03 : rq47) >> (8 * (i & 3))) & 0xFFu) : 0u;
    const bool lane_ok = L < (1u << nl);
    const uint32_t jmax = 1u << nr;
    const bool init = src_s == kInit;
    const cplx<R> *src = a.states + (uint64_t)(init ? 0u : src_s) * a.slot_amps + base;

    // a full tile (64 lanes, RB register qubits) loads without predication:
    // scalar base of each register index plus the lane offset
    const bool full = nl == kLaneBits && nr == (uint32_t)RB;
    // (branches sit outside the unrolled loops so all loads issue back to back)
    auto reg_off = [&](auto Jc) __attribute__((always_inline)) {
        constexpr int j = decltype(Jc)::value;
        uint32_t off = 0;
        sfor<RB>([&](auto Ic) __attribute__((always_inline)) {
            constexpr int i = decltype(Ic)::value;
            if constexpr ((j >> i) & 1) off |= 1u << rq[i];
        });
        return off;
    };
    cplx<R> v[NJ];
    if (init) {
        sfor<NJ>([&](auto Jc) __attribute__((always_inline)) {
            constexpr int j = decltype(Jc)::value;
            const uint32_t off = reg_off(Jc);
            v[j] = cplx<R>{(uint32_t)j < jmax && (base + off + L) == 0 ? R(1) : R(0), R(0)};
        });
    } else if (full) {
        sfor<NJ>([&](auto Jc) __attribute__((always_inline)) {
            constexpr int j = decltype(Jc)::value;
            v[j] = (src + reg_off(Jc))[L];
        });
    } else {
        sfor<NJ>([&](auto Jc) __attribute__((always_inline)) {
            constexpr int j = decltype(Jc)::value;
            v[j] = cplx<R>{R(0), R(0)};
            if ((uint32_t)j < jmax && lane_ok) v[j] = (src + reg_off(Jc))[L];
        });
    }

    // frame at the start of this pass
    const uint32_t node = kconst(a.node_ids)[traj];
    uint32_t fx = kconst(a.meta.frame0)[2 * node], fz = kconst(a.meta.frame0)[2 * node + 1];
    uint32_t e = kconst(a.meta.ev_off)[node];
    const uint32_t e1 = kconst(a.meta.ev_off)[node + 1];
    while (e < e1 && ev_pos[e] < a.pass_key) {
        fx ^= ev_dx[e];
        fz ^= ev_dz[e];
        e++;
    }

    for (uint32_t oi = 0; oi < op_count; oi++) {
        const OpDesc o = kload(ops + op_begin + oi);
        while (e < e1 && ev_pos[e] <= (a.pass_key | o.slot0)) {
            fx ^= ev_dx[e];
            fz ^= ev_dz[e];
            e++;
        }
        if (o.kind == OP_DIAGRUN) {
            const bool inside = e < e1 && ev_pos[e] < (a.pass_key | o.slot1);
            if (!inside) {
                op_diag_run<R, RB>(v, o, mats + o.mat, kconst(a.terms) + o.terms, fx, L, base, rq, nr);
                continue;
            }
            // events inside the run (counted up to four)
            const uint32_t end = a.pass_key | o.slot1;
            uint32_t ne = 1;
            while (ne < 4u && e + ne < e1 && ev_pos[e + ne] < end) ne++;
            if (o.ngates < 255u && ne <= 3u) {
                // up to three: the run in up to four frames, the gates on
                // register qubits only one by one (event indexes stay in
                // [e, e1))
                const uint32_t eb = ne > 1u ? e + 1 : e, ec = ne > 2u ? e + 2 : eb;
                RunFrames rf;
                rf.f0 = fx;
                rf.k0 = (ev_pos[e] & 0xFFFFu) - o.slot0;
                rf.f1 = fx ^ ev_dx[e];
                rf.k1 = ne > 1u ? (ev_pos[eb] & 0xFFFFu) - o.slot0 : 255u;
                rf.f2 = ne > 1u ? rf.f1 ^ ev_dx[eb] : rf.f1;
                rf.k2 = ne > 2u ? (ev_pos[ec] & 0xFFFFu) - o.slot0 : 255u;
                rf.f3 = ne > 2u ? rf.f2 ^ ev_dx[ec] : rf.f2;
                op_diag_run_split<R, RB>(v, o, kconst(a.terms) + o.terms, rf, L, base, rq);
                if (o.has_t) {
                    for (uint32_t k = 0; k < o.ngates; k++) {
                        const DiagGate dg = kload(kconst(a.dgates) + o.gates + k);
                        const bool regonly = dg.role[0] == ROLE_REG && (dg.nq == 1 || dg.role[1] == ROLE_REG);
                        if (regonly) op_diag_one<R, RB>(v, dg, mats + dg.d, rf.at(k), L, base);
                    }
                }
                fx = rf.f3;
                fz ^= ev_dz[e] ^ (ne > 1u ? ev_dz[eb] : 0u) ^ (ne > 2u ? ev_dz[ec] : 0u);
                e += ne;
            } else {
                // more events inside the run: gate by gate with frame updates
                for (uint32_t k = 0; k < o.ngates; k++) {
                    while (e < e1 && ev_pos[e] <= (a.pass_key | (o.slot0 + k))) {
                        fx ^= ev_dx[e];
                        fz ^= ev_dz[e];
                        e++;
                    }
                    const DiagGate dg = kload(kconst(a.dgates) + o.gates + k);
                    op_diag_one<R, RB>(v, dg, mats + dg.d, fx, L, base);
                }
            }
            continue;
        }
        uint32_t xl = (fx >> o.phys[0]) & 1u, zl = (fz >> o.phys[0]) & 1u;
        if (o.nq == 2) {
            xl |= ((fx >> o.phys[1]) & 1u) << 1;
            zl |= ((fz >> o.phys[1]) & 1u) << 1;
        }
        const kptr<cplx<R>> G = mats + o.mat;
        if constexpr (D2) {
            if (o.kind == OP_DENSE2) {
                op_dense2<R, RB>(v, o, G, xl, zl, L);
                continue;
            }
        }
        op_dense1<R, RB>(v, o, G, xl, zl, L, base);
    }

    cplx<R> *dst = a.states + (uint64_t)dst_s * a.slot_amps + base;
    if (full) {
        sfor<NJ>([&](auto Jc) __attribute__((always_inline)) {
            constexpr int j = decltype(Jc)::value;
            (dst + reg_off(Jc))[L] = v[j];
        });
    } else {
        sfor<NJ>([&](auto Jc) __attribute__((always_inline)) {
            constexpr int j = decltype(Jc)::value;
            if ((uint32_t)j < jmax && lane_ok) (dst + reg_off(Jc))[L] = v[j];
        });
    }
    if (a.part && full) tile_partials<R, RB>(v, a, traj, tile, nfree, L);
}

}  // namespace tqs
