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

#include "tile_common.h"

namespace tqs {

// ---------------------------------------------------------------- DENSE1 --
// 2x2 on the target qubit; with nq == 2 the gate is block-diagonal in the
// other (control) qubit and the control's value selects the block.
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
    const uint32_t traj = a.perm ? kconst(a.perm)[w % a.count] : w % a.count, tile = w / a.count;
    const uint32_t L = threadIdx.x;
    const kptr<PassDesc> pd = kconst(a.pass);
    const kptr<OpDesc> ops = kconst(a.ops);
    const kptr<cplx<R>> mats = kconst(a.mats);
    const kptr<uint32_t> ev_pos = kconst(a.meta.ev_pos), ev_dx = kconst(a.meta.ev_dx),
                         ev_dz = kconst(a.meta.ev_dz);
    static_assert(__builtin_offsetof(PassDesc, nl) == 8 && __builtin_offsetof(PassDesc, rq) == 12 &&
                      __builtin_offsetof(PassDesc, fbits) == 20,
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

// ------------------------------------------------------- level pass tile --
// One pass of the level kernel over one tile of one trajectory (traj: index
// in the launched chunk): the body of pass_kernel, with the tile read from
// the state in LDS (from_lds; physical amplitude order) instead of HBM, and
// written back to LDS (to_lds) instead of HBM.  (pass_kernel keeps its own
// copy: factored into a shared function, its register allocation spills
// several times more.)
template <typename R, int RB, bool D2>
__device__ __forceinline__ void level_pass_tile(const PassArgs<R> &a, uint32_t traj, uint32_t tile, uint32_t L,
                                          cplx<R> *st, bool from_lds, bool to_lds) {
    constexpr int NJ = 1 << RB;
    const kptr<PassDesc> pd = kconst(a.pass);
    const kptr<OpDesc> ops = kconst(a.ops);
    const kptr<cplx<R>> mats = kconst(a.mats);
    const kptr<uint32_t> ev_pos = kconst(a.meta.ev_pos), ev_dx = kconst(a.meta.ev_dx),
                         ev_dz = kconst(a.meta.ev_dz);
    static_assert(__builtin_offsetof(PassDesc, nl) == 8 && __builtin_offsetof(PassDesc, rq) == 12 &&
                      __builtin_offsetof(PassDesc, fbits) == 20,
                  "pass descriptor layout");
    const kptr<uint32_t> pw = (kptr<uint32_t>)pd;
    const uint32_t op_begin = uni(pw[0]), op_count = uni(pw[1]), pw2 = uni(pw[2]);
    const uint32_t rq03 = uni(pw[3]), rq47 = uni(pw[4]);
    const uint32_t nl = pw2 & 0xFFu, nr = (pw2 >> 8) & 0xFFu, nfree = (pw2 >> 16) & 0xFFu;
    if (tile >> nfree) return;  // (a workgroup wider than this pass's tile count)

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
    if (from_lds) {
        // the state in LDS (physical order), left there by the previous pass
        sfor<NJ>([&](auto Jc) __attribute__((always_inline)) {
            constexpr int j = decltype(Jc)::value;
            v[j] = cplx<R>{R(0), R(0)};
            if (full || ((uint32_t)j < jmax && lane_ok)) v[j] = st[base + reg_off(Jc) + L];
        });
    } else if (init) {
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

    if (to_lds) {
        sfor<NJ>([&](auto Jc) __attribute__((always_inline)) {
            constexpr int j = decltype(Jc)::value;
            if (full || ((uint32_t)j < jmax && lane_ok)) st[base + reg_off(Jc) + L] = v[j];
        });
        return;
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

// ----------------------------------------------------------- level kernel --
// Every pass of one tree level over a chunk of states small enough for LDS
// (2^n amplitudes in one workgroup's LDS): one workgroup per state, one wave
// per tile.  The first pass reads the parent's state from HBM (or makes
// |0..0>), later passes read what the previous one left in LDS, and only
// the last writes to HBM (with the sampling partials at the leaf level), so
// a level costs one launch and one read and write of each state instead of
// one of each per pass.
constexpr uint32_t kLevelThreads = 512;  // up to eight tiles per state

template <typename R>
struct LevelLaunch {
    PassArgs<R> a;   // the level's first pass, for the chunk's computed states
    uint32_t npass;  // its passes: descriptors a.pass[0, npass), keys a.pass_key + (k << 16)
    uint32_t psum;   // partial-sum layout of the last pass
    double *part;    // sampling partials the last pass writes (or NULL)
};

template <typename R, int RB, bool D2>
__global__ __launch_bounds__(kLevelThreads, 2) void level_kernel(LevelLaunch<R> ll) {
    extern __shared__ unsigned char level_lds[];
    cplx<R> *st = reinterpret_cast<cplx<R> *>(level_lds);
    const uint32_t nwg = gridDim.x, bid = blockIdx.x;
    const uint32_t ti = (bid & 7u) * (nwg >> 3) + (bid >> 3);
    if (ti >= ll.a.count) return;  // (the whole workgroup)
    const uint32_t tv = threadIdx.x >> 6, L = threadIdx.x & 63u;
    PassArgs<R> a = ll.a;
    for (uint32_t k = 0; k < ll.npass; k++) {
        if (k) {
            __syncthreads();
            a.pass = ll.a.pass + k;
            a.pass_key = ll.a.pass_key + (k << 16);
        }
        const bool last = k + 1 == ll.npass;
        a.part = last ? ll.part : nullptr;
        a.psum = last ? ll.psum : 0u;
        level_pass_tile<R, RB, D2>(a, ti, tv, L, st, k > 0, !last);
    }
}

}  // namespace tqs
