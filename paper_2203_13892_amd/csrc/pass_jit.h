// Building blocks of plan-specialised pass kernels, compiled at run time
// (hipRTC) from source the planner writes for each pass of a plan.
//
// The tile is the one of pass_kernel.h: one wave per workgroup, one tile of
// one trajectory, lane L holding the amplitudes whose low physical qubits
// spell L and register index j spelling the register qubits.  Here every
// op's kind, qubit roles and positions, and every phase term's qubits and
// phases are compile-time constants, so a pass is straight-line code: no
// per-op descriptor reads or dispatch, and the tile stays in the same
// registers from op to op.  Only the trajectory's Pauli frame and noise
// events are read at run time (wave-uniform, scalar unit).
//
// Phase runs: each term's phases are re-indexed by its frame bits and
// split into the multilinear coefficients of its two index bits,
//   th(y_u, y_w) = a + b x_u + g x_w + d x_u x_w   (x: stored index bits),
// accumulated per run on the scalar unit into a constant, per-lane-bit and
// lane-pair coefficients, and per-register-bit coefficients; each lane then
// evaluates its phase from its own bits.  Gates on register qubits only
// form the run's table T (host side), read at index j ^ (frame's register
// bits) when they all see one frame; nodes whose frame changes between
// them take the generic pass kernel instead (the executor routes them).
#pragma once

#include "tile_common.h"

namespace tqs {
namespace jit {

constexpr int kNone = 3;  // no control qubit (one-qubit gate)

// Wave state: tile origin, the trajectory's Pauli frame and the cursor over
// its node's noise events (keys (pass << 16) | gate slot).
struct Wave {
    uint32_t L, base;
    uint32_t fx, fz;
    uint32_t e, e1, nxt;
    kptr<uint32_t> pos, dx, dz;
};

// Apply the events up to key (those acting before the op at this slot).
__device__ __forceinline__ void advance(Wave &w, uint32_t key) {
    while (w.nxt <= key) {
        w.fx ^= uni(w.dx[w.e]);
        w.fz ^= uni(w.dz[w.e]);
        w.e++;
        w.nxt = w.e < w.e1 ? uni(w.pos[w.e]) : 0xFFFFFFFFu;
    }
}

// Frame bits of one or two qubits as a local index (bit 0: first qubit).
__device__ __forceinline__ uint32_t local2(uint32_t f, uint32_t p0, uint32_t p1, uint32_t nq) {
    uint32_t x = (f >> p0) & 1u;
    if (nq == 2) x |= ((f >> p1) & 1u) << 1;
    return x;
}

// Value of the lane whose index differs in the bits of M: quad permutes
// for masks below 4, the 32-lane swizzle below 32, a permute otherwise.
template <int M>
__device__ __forceinline__ int lane_xor_i(int i) {
    static_assert(M > 0 && M < 64, "lane mask");
    // (quad permutes read a valid lane everywhere: bound_ctrl, no old value)
    if constexpr (M == 1) return __builtin_amdgcn_mov_dpp(i, 0xB1, 0xF, 0xF, true);
    else if constexpr (M == 2) return __builtin_amdgcn_mov_dpp(i, 0x4E, 0xF, 0xF, true);
    else if constexpr (M == 3) return __builtin_amdgcn_mov_dpp(i, 0x1B, 0xF, 0xF, true);
    else if constexpr (M < 32) return __builtin_amdgcn_ds_swizzle(i, (M << 10) | 0x1F);
    else return __builtin_amdgcn_ds_bpermute((int)(((uint32_t)__lane_id() ^ (uint32_t)M) << 2), i);
}
template <int M>
__device__ __forceinline__ float lane_xor(float x) {
    return __int_as_float(lane_xor_i<M>(__float_as_int(x)));
}
template <int M>
__device__ __forceinline__ double lane_xor(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = lane_xor_i<M>((int)(b & 0xFFFFFFFFll)), hi = lane_xor_i<M>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(uint32_t)lo);
}
template <int M, typename R>
__device__ __forceinline__ cplx<R> lane_xor_c(cplx<R> v) {
    return {lane_xor<M>(v.re), lane_xor<M>(v.im)};
}

// Keeps an updated amplitude's arithmetic where it is written: without it
// the multiply-adds can sink past later cross-lane reads, which then all
// hold their results at once (register spills).  No instruction is emitted.
template <typename R>
__device__ __forceinline__ void pin(cplx<R> &v) {
    asm volatile("" : "+v"(v.re), "+v"(v.im));
}

// ------------------------------------------------------------ dense 2x2 --
// A 2x2 gate on qubit TPOS (lane bit or register bit), or a two-qubit gate
// block-diagonal in its control qubit (role CROLE at CPOS; kNone for a
// one-qubit gate).  TQ: which of the gate's two qubits is the target.
template <typename R, int RB, bool REAL, int TROLE, int TPOS, int CROLE, int CPOS, int NQ, int TQ>
__device__ __forceinline__ void d1(cplx<R> (&v)[1 << RB], kptr<cplx<R>> G, uint32_t xl, uint32_t zl,
                                   const Wave &w) {
    constexpr int NJ = 1 << RB;
    constexpr uint32_t K = 1u << NQ, CQ = 1u - (uint32_t)TQ;
    cplx<R> B[2][4];
#pragma unroll
    for (uint32_t cb = 0; cb < 2; cb++)
#pragma unroll
        for (uint32_t rr = 0; rr < 2; rr++)
#pragma unroll
            for (uint32_t cc = 0; cc < 2; cc++) {
                uint32_t r = rr << TQ, c = cc << TQ;
                if constexpr (NQ == 2) {
                    r |= cb << CQ;
                    c |= cb << CQ;
                }
                B[cb][rr * 2 + cc] = conj_entry(G, K, r, c, xl, zl);
            }
    if constexpr (TROLE == ROLE_REG) {
        if constexpr (CROLE == ROLE_REG) {
            sfor<NJ>([&](auto Jc) __attribute__((always_inline)) {
                constexpr int j = decltype(Jc)::value;
                if constexpr (!(j & (1 << TPOS))) {
                    constexpr int cb = (j >> CPOS) & 1;
                    const cplx<R> x0 = v[j], x1 = v[j | (1 << TPOS)];
                    v[j] = mmac<REAL>(mmul<REAL>(B[cb][0], x0), B[cb][1], x1);
                    v[j | (1 << TPOS)] = mmac<REAL>(mmul<REAL>(B[cb][2], x0), B[cb][3], x1);
                }
            });
        } else {
            cplx<R> M[4];
            if constexpr (CROLE == ROLE_LANE) {
                const bool cb = ((w.L >> CPOS) & 1u) != 0;
#pragma unroll
                for (int e = 0; e < 4; e++) M[e] = csel(cb, B[1][e], B[0][e]);
            } else if constexpr (CROLE == ROLE_FIXED) {
                const bool cb = ((w.base >> CPOS) & 1u) != 0;
#pragma unroll
                for (int e = 0; e < 4; e++) M[e] = csel(cb, B[1][e], B[0][e]);
            } else {
#pragma unroll
                for (int e = 0; e < 4; e++) M[e] = B[0][e];
            }
            sfor<NJ>([&](auto Jc) __attribute__((always_inline)) {
                constexpr int j = decltype(Jc)::value;
                if constexpr (!(j & (1 << TPOS))) {
                    const cplx<R> x0 = v[j], x1 = v[j | (1 << TPOS)];
                    v[j] = mmac<REAL>(mmul<REAL>(M[0], x0), M[1], x1);
                    v[j | (1 << TPOS)] = mmac<REAL>(mmul<REAL>(M[2], x0), M[3], x1);
                }
            });
        }
    } else {
        // lane target: own row b, partner (lane ^ 2^TPOS) in column 1 - b
        const bool b = ((w.L >> TPOS) & 1u) != 0;
        if constexpr (CROLE == ROLE_REG) {
            const cplx<R> a0 = csel(b, B[0][3], B[0][0]), c0 = csel(b, B[0][2], B[0][1]);
            const cplx<R> a1 = csel(b, B[1][3], B[1][0]), c1 = csel(b, B[1][2], B[1][1]);
            sfor<NJ>([&](auto Jc) __attribute__((always_inline)) {
                constexpr int j = decltype(Jc)::value;
                constexpr int cb = (j >> CPOS) & 1;
                const cplx<R> p = lane_xor_c<1 << TPOS>(v[j]);
                v[j] = mmac<REAL>(mmul<REAL>(cb ? a1 : a0, v[j]), cb ? c1 : c0, p);
                pin(v[j]);
                shuffle_fence<j>();
            });
        } else {
            bool cb = false;
            if constexpr (CROLE == ROLE_LANE) cb = ((w.L >> CPOS) & 1u) != 0;
            else if constexpr (CROLE == ROLE_FIXED) cb = ((w.base >> CPOS) & 1u) != 0;
            const cplx<R> a = csel(b, csel(cb, B[1][3], B[0][3]), csel(cb, B[1][0], B[0][0]));
            const cplx<R> c = csel(b, csel(cb, B[1][2], B[0][2]), csel(cb, B[1][1], B[0][1]));
            sfor<NJ>([&](auto Jc) __attribute__((always_inline)) {
                constexpr int j = decltype(Jc)::value;
                const cplx<R> p = lane_xor_c<1 << TPOS>(v[j]);
                v[j] = mmac<REAL>(mmul<REAL>(a, v[j]), c, p);
                pin(v[j]);
                shuffle_fence<j>();
            });
        }
    }
}

// ---------------------------------------------------------- butterflies --
// A one-qubit gate whose four entries are +-s (a Hadamard up to signs), as
// the butterfly out_r = sum_c sigma_rc x_c without its common factor s: the
// pass multiplies the tile by the product of these factors once, before it
// stores it (scale_tile).  NEG: bit 2r + c set where sigma_rc = -1.  The
// frame on the qubit conjugates the signs as conj_entry does a matrix,
// sigma'_rc = sigma_{r^x, c^x} (-1)^{z r + z c}.
template <int NEG, int RR, int CC>
struct Sgn {
    static constexpr int value = ((NEG >> (2 * RR + CC)) & 1) ? -1 : 1;
};

template <int NEG, typename R>
__device__ __forceinline__ R conj_sign(uint32_t r, uint32_t c, uint32_t xl, uint32_t zl) {
    const uint32_t flip = ((uint32_t)(NEG >> (2 * (r ^ xl) + (c ^ xl))) & 1u) ^ ((zl & r) ^ (zl & c));
    return flip ? R(-1) : R(1);
}

// Register target: one add or subtract per real output with no frame on
// the qubit (signs known when the pass is compiled), a multiply and a
// multiply-add with one (signs from the frame).
template <typename R, int RB, int TPOS, int NEG>
__device__ __forceinline__ void bf_reg(cplx<R> (&v)[1 << RB], uint32_t xl, uint32_t zl) {
    constexpr int NJ = 1 << RB;
    if ((xl | zl) == 0) {
        constexpr int s00 = Sgn<NEG, 0, 0>::value, s01 = Sgn<NEG, 0, 1>::value;
        constexpr int s10 = Sgn<NEG, 1, 0>::value, s11 = Sgn<NEG, 1, 1>::value;
        sfor<NJ>([&](auto Jc) __attribute__((always_inline)) {
            constexpr int j = decltype(Jc)::value;
            if constexpr (!(j & (1 << TPOS))) {
                const cplx<R> x0 = v[j], x1 = v[j | (1 << TPOS)];
                v[j] = {R(s00) * x0.re + R(s01) * x1.re, R(s00) * x0.im + R(s01) * x1.im};
                v[j | (1 << TPOS)] = {R(s10) * x0.re + R(s11) * x1.re, R(s10) * x0.im + R(s11) * x1.im};
            }
        });
    } else {
        const R S0 = conj_sign<NEG, R>(0, 0, xl, zl), S1 = conj_sign<NEG, R>(0, 1, xl, zl);
        const R S2 = conj_sign<NEG, R>(1, 0, xl, zl), S3 = conj_sign<NEG, R>(1, 1, xl, zl);
        sfor<NJ>([&](auto Jc) __attribute__((always_inline)) {
            constexpr int j = decltype(Jc)::value;
            if constexpr (!(j & (1 << TPOS))) {
                const cplx<R> x0 = v[j], x1 = v[j | (1 << TPOS)];
                v[j] = {S0 * x0.re + S1 * x1.re, S0 * x0.im + S1 * x1.im};
                v[j | (1 << TPOS)] = {S2 * x0.re + S3 * x1.re, S2 * x0.im + S3 * x1.im};
            }
        });
    }
}

// Lane target: own row b (own value in column b, the partner's in column
// 1 - b), out = a x_own + c x_partner with a, c = +-1 per lane.  Written as
// a (x_own + a c x_partner): one multiply-add per real output (the
// partner's value feeds it straight from the quad permute, swizzle or
// permute), and the per-lane sign a joins `sg`, the tile's deferred
// per-lane sign.  That sign depends on lane bit TPOS only, so it commutes
// with every later op that does not mix that bit (diagonal runs, register
// ops, ops on other lane bits, ops controlled by it); the pass applies it
// with the common factors before the store, or earlier (flush_sign) before
// an op that mixes the bit.  The products are exact, so the results are
// those of a x_own + c x_partner rounded once.
template <typename R, int RB, int TPOS, int NEG>
__device__ __forceinline__ void bf_lane(cplx<R> (&v)[1 << RB], uint32_t xl, uint32_t zl, const Wave &w, R &sg) {
    constexpr int NJ = 1 << RB;
    const bool b = ((w.L >> TPOS) & 1u) != 0;
    const R a = b ? conj_sign<NEG, R>(1, 1, xl, zl) : conj_sign<NEG, R>(0, 0, xl, zl);
    const R k = a * (b ? conj_sign<NEG, R>(1, 0, xl, zl) : conj_sign<NEG, R>(0, 1, xl, zl));
    sfor<NJ>([&](auto Jc) __attribute__((always_inline)) {
        constexpr int j = decltype(Jc)::value;
        const cplx<R> p = lane_xor_c<1 << TPOS>(v[j]);
        v[j] = {v[j].re + k * p.re, v[j].im + k * p.im};
        pin(v[j]);
        shuffle_fence<j>();
    });
    sg *= a;
}

// The deferred per-lane sign applied now (before an op that mixes a lane
// bit it depends on).
template <typename R, int RB>
__device__ __forceinline__ void flush_sign(cplx<R> (&v)[1 << RB], R &sg) {
    sfor<(1 << RB)>([&](auto Jc) __attribute__((always_inline)) {
        constexpr int j = decltype(Jc)::value;
        v[j] = {v[j].re * sg, v[j].im * sg};
    });
    sg = R(1);
}

// The tile times a real factor (the butterflies' common factors, with the
// deferred per-lane sign).
template <typename R, int RB>
__device__ __forceinline__ void scale_tile(cplx<R> (&v)[1 << RB], R s) {
    sfor<(1 << RB)>([&](auto Jc) __attribute__((always_inline)) {
        constexpr int j = decltype(Jc)::value;
        v[j] = {v[j].re * s, v[j].im * s};
    });
}

// ------------------------------------------------------------ dense 4x4 --
// A two-qubit gate on qubits (P0, P1) in normalised order: the first is a
// register qubit whenever one of them is, and register pairs have P0 < P1.
// SW: the gate's own qubit order is the reverse of the normalised one.
template <typename R, int RB, bool SW, bool REG0, bool REG1, int P0, int P1>
__device__ __forceinline__ void d2(cplx<R> (&v)[1 << RB], kptr<cplx<R>> G, uint32_t xl, uint32_t zl,
                                   const Wave &w) {
    constexpr int NJ = 1 << RB;
    cplx<R> M[16];
#pragma unroll
    for (uint32_t r = 0; r < 4; r++)
#pragma unroll
        for (uint32_t c = 0; c < 4; c++) {
            const uint32_t rs = SW ? ((r >> 1) | ((r & 1u) << 1)) : r;
            const uint32_t cs = SW ? ((c >> 1) | ((c & 1u) << 1)) : c;
            M[r * 4 + c] = conj_entry(G, 4, rs, cs, xl, zl);
        }
    if constexpr (REG0 && REG1) {
        static_assert(P0 < P1, "normalised register pair");
        sfor<NJ>([&](auto Jc) __attribute__((always_inline)) {
            constexpr int j = decltype(Jc)::value;
            if constexpr (!(j & ((1 << P0) | (1 << P1)))) {
                constexpr int i0 = j, i1 = j | (1 << P0), i2 = j | (1 << P1), i3 = j | (1 << P0) | (1 << P1);
                const cplx<R> x0 = v[i0], x1 = v[i1], x2 = v[i2], x3 = v[i3];
                v[i0] = cmac(cmac(cmac(cmul(M[0], x0), M[1], x1), M[2], x2), M[3], x3);
                v[i1] = cmac(cmac(cmac(cmul(M[4], x0), M[5], x1), M[6], x2), M[7], x3);
                v[i2] = cmac(cmac(cmac(cmul(M[8], x0), M[9], x1), M[10], x2), M[11], x3);
                v[i3] = cmac(cmac(cmac(cmul(M[12], x0), M[13], x1), M[14], x2), M[15], x3);
            }
            shuffle_fence<j>();
        });
    } else if constexpr (REG0) {
        // register bit P0, lane bit P1: own rows 2b, 2b+1; partner columns
        const bool b = ((w.L >> P1) & 1u) != 0;
        cplx<R> k0[4], k1[4];
#pragma unroll
        for (uint32_t cc = 0; cc < 4; cc++) {
            // (own a0, own a1, partner q0, partner q1) are columns cc for
            // b = 0 and cc ^ 2 for b = 1
            k0[cc] = csel(b, M[2 * 4 + (cc ^ 2u)], M[0 * 4 + cc]);
            k1[cc] = csel(b, M[3 * 4 + (cc ^ 2u)], M[1 * 4 + cc]);
        }
        sfor<NJ>([&](auto Jc) __attribute__((always_inline)) {
            constexpr int j = decltype(Jc)::value;
            if constexpr (!(j & (1 << P0))) {
                const cplx<R> a0 = v[j], a1 = v[j | (1 << P0)];
                const cplx<R> q0 = lane_xor_c<1 << P1>(a0), q1 = lane_xor_c<1 << P1>(a1);
                v[j] = cmac(cmac(cmac(cmul(k0[0], a0), k0[1], a1), k0[2], q0), k0[3], q1);
                v[j | (1 << P0)] = cmac(cmac(cmac(cmul(k1[0], a0), k1[1], a1), k1[2], q0), k1[3], q1);
                pin(v[j]);
                pin(v[j | (1 << P0)]);
            }
            shuffle_fence<j>();
        });
    } else {
        // both on lanes: own index r = b0 + 2 b1, partners r ^ 1, r ^ 2, r ^ 3
        const uint32_t r = ((w.L >> P0) & 1u) | (((w.L >> P1) & 1u) << 1);
        cplx<R> k[4];
#pragma unroll
        for (uint32_t d = 0; d < 4; d++) {
            const cplx<R> e0 = M[0 * 4 + (0 ^ d)], e1 = M[1 * 4 + (1 ^ d)];
            const cplx<R> e2 = M[2 * 4 + (2 ^ d)], e3 = M[3 * 4 + (3 ^ d)];
            k[d] = csel(r == 3, e3, csel(r == 2, e2, csel(r == 1, e1, e0)));
        }
        sfor<NJ>([&](auto Jc) __attribute__((always_inline)) {
            constexpr int j = decltype(Jc)::value;
            const cplx<R> q1 = lane_xor_c<1 << P0>(v[j]);
            const cplx<R> q2 = lane_xor_c<1 << P1>(v[j]);
            const cplx<R> q3 = lane_xor_c<(1 << P0) | (1 << P1)>(v[j]);
            v[j] = cmac(cmac(cmac(cmul(k[0], v[j]), k[1], q1), k[2], q2), k[3], q3);
            pin(v[j]);
            shuffle_fence<j>();
        });
    }
}

// ------------------------------------------------------ fused 32x32 (MFMA) --
// A unitary on the tile's five register qubits (complex64), fused from
// consecutive register-only dense ops, applied on the matrix cores with
// v_mfma_f32_32x32x2_f32.  Out = U_F V with V the tile as a 32 x 64 matrix
// (register index x lane) and U_F = F^dagger U F for the frame's register
// bits (x, z): U_F[r][c] = U[r ^ x][c ^ x] (-1)^{z.r + z.c}.
//   B operand (K = 2, N = 32): lane l holds B[l / 32][l % 32].  Swapping
//   the upper lanes of register 2s with the lower lanes of register 2s+1
//   (v_permlane32_swap) gives the operands of input rows (2s, 2s+1) for
//   columns 0-31 and 32-63.
//   A operand (M = 32, K = 2): lane l holds A[l % 32][l / 32], i.e.
//   U_F[l % 32][2s + l / 32], read from the plan's row-major U.
//   Result: accumulator r of lane l is row 8 (r / 4) + 4 (l / 32) + r % 4 of
//   column l % 32; swapping the halves of the two column blocks' registers
//   puts every lane's own column back in its registers.
// Complex products as four real ones per step: re += Ur Vr - Ui Vi,
// im += Ur Vi + Ui Vr.  128 MFMAs, 64 lane swaps and 16 loads per lane.
typedef float mfma_v16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ void mfma32(cplx<float> (&v)[32], kptr<cplx<float>> U, uint32_t x, uint32_t z,
                                       uint32_t L) {
    const uint32_t m = L & 31u, h = L >> 5;
    const uint32_t row = (m ^ x) * 32u;
    const uint32_t sr = (uint32_t)__builtin_popcount(z & m) & 1u;
    // the lane's A entries for the 16 K steps (loads first)
    cplx<float> a[16];
#pragma unroll
    for (uint32_t s = 0; s < 16; s++) a[s] = U[row + ((2u * s + h) ^ x)];
    // B operands
    uint32_t br[32], bi[32];
#pragma unroll
    for (uint32_t s = 0; s < 16; s++) {
        const auto pr = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[2 * s].re), __float_as_uint(v[2 * s + 1].re),
                                                         false, false);
        const auto pi = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[2 * s].im), __float_as_uint(v[2 * s + 1].im),
                                                         false, false);
        br[2 * s] = pr[0];
        br[2 * s + 1] = pr[1];
        bi[2 * s] = pi[0];
        bi[2 * s + 1] = pi[1];
    }
    mfma_v16 re0 = {0}, im0 = {0}, re1 = {0}, im1 = {0};
#pragma unroll
    for (uint32_t s = 0; s < 16; s++) {
        // frame signs of entry (m, 2s + h)
        const uint32_t sg = (sr ^ ((uint32_t)__builtin_popcount(z & (2u * s + h)) & 1u)) << 31;
        const float ar = __uint_as_float(__float_as_uint(a[s].re) ^ sg);
        const float ai = __uint_as_float(__float_as_uint(a[s].im) ^ sg);
        const float an = -ai;
        const float b0r = __uint_as_float(br[2 * s]), b0i = __uint_as_float(bi[2 * s]);
        const float b1r = __uint_as_float(br[2 * s + 1]), b1i = __uint_as_float(bi[2 * s + 1]);
        re0 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, b0r, re0, 0, 0, 0);
        re0 = __builtin_amdgcn_mfma_f32_32x32x2f32(an, b0i, re0, 0, 0, 0);
        im0 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, b0i, im0, 0, 0, 0);
        im0 = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, b0r, im0, 0, 0, 0);
        re1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, b1r, re1, 0, 0, 0);
        re1 = __builtin_amdgcn_mfma_f32_32x32x2f32(an, b1i, re1, 0, 0, 0);
        im1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, b1i, im1, 0, 0, 0);
        im1 = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, b1r, im1, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 16; r++) {
        const auto qr = __builtin_amdgcn_permlane32_swap(__float_as_uint(re0[r]), __float_as_uint(re1[r]), false, false);
        const auto qi = __builtin_amdgcn_permlane32_swap(__float_as_uint(im0[r]), __float_as_uint(im1[r]), false, false);
        const int lo = 8 * (r / 4) + r % 4;
        v[lo] = cplx<float>{__uint_as_float(qr[0]), __uint_as_float(qi[0])};
        v[lo + 4] = cplx<float>{__uint_as_float(qr[1]), __uint_as_float(qi[1])};
    }
}

// ------------------------------------------------------------ phase runs --
// Events strictly inside a run (at most three; the executor routes nodes
// with more to the generic kernel): the frame a gate of the run sees, by
// its index k in the run.  Consumes the events and leaves the frame at the
// run's end.
__device__ __forceinline__ RunFrames run_frames(Wave &w, uint32_t key0, uint32_t key1) {
    RunFrames rf;
    rf.f0 = rf.f1 = rf.f2 = rf.f3 = w.fx;
    rf.k0 = rf.k1 = rf.k2 = 0xFFFFu;
    if (w.nxt < key1) {
        rf.k0 = (w.nxt & 0xFFFFu) - (key0 & 0xFFFFu);
        rf.f1 = rf.f0 ^ uni(w.dx[w.e]);
        w.fz ^= uni(w.dz[w.e]);
        w.e++;
        w.nxt = w.e < w.e1 ? uni(w.pos[w.e]) : 0xFFFFFFFFu;
        rf.f2 = rf.f3 = rf.f1;
        if (w.nxt < key1) {
            rf.k1 = (w.nxt & 0xFFFFu) - (key0 & 0xFFFFu);
            rf.f2 = rf.f1 ^ uni(w.dx[w.e]);
            w.fz ^= uni(w.dz[w.e]);
            w.e++;
            w.nxt = w.e < w.e1 ? uni(w.pos[w.e]) : 0xFFFFFFFFu;
            rf.f3 = rf.f2;
            if (w.nxt < key1) {
                rf.k2 = (w.nxt & 0xFFFFu) - (key0 & 0xFFFFu);
                rf.f3 = rf.f2 ^ uni(w.dx[w.e]);
                w.fz ^= uni(w.dz[w.e]);
                w.e++;
                w.nxt = w.e < w.e1 ? uni(w.pos[w.e]) : 0xFFFFFFFFu;
            }
        }
    }
    w.fx = rf.f3;
    return rf;
}

// One term's four phases re-indexed by its frame bits (fu, fw) and split
// into multilinear coefficients of the stored index bits (x_u, x_w):
// th(x_u ^ fu, x_w ^ fw) = a + b x_u + g x_w + d x_u x_w  (mod one turn).
template <typename A>
struct Ml {
    A a, b, g, d;
};
template <typename A>
__device__ __forceinline__ Ml<A> multilinear(A t0, A t1, A t2, A t3, uint32_t fu, uint32_t fw) {
    // permute by the frame: index (x_u ^ fu) + 2 (x_w ^ fw)
    const A u0 = fu ? t1 : t0, u1 = fu ? t0 : t1, u2 = fu ? t3 : t2, u3 = fu ? t2 : t3;
    const A p0 = fw ? u2 : u0, p1 = fw ? u3 : u1, p2 = fw ? u0 : u2, p3 = fw ? u1 : u3;
    Ml<A> m;
    m.a = p0;
    m.b = (A)(p1 - p0);
    m.g = (A)(p2 - p0);
    m.d = (A)(p3 - p2 - p1 + p0);
    return m;
}

// Per-lane masks of the lane bits: all ones where bit a of L is set.
struct LaneBits {
    uint32_t m[6];
};
__device__ __forceinline__ LaneBits lane_bits(uint32_t L) {
    LaneBits lb;
#pragma unroll
    for (int a = 0; a < 6; a++) lb.m[a] = 0u - ((L >> a) & 1u);
    return lb;
}
// c where the mask is set (per lane), in the accumulator width
__device__ __forceinline__ uint32_t masked(uint32_t c, uint32_t m) { return c & m; }
__device__ __forceinline__ uint64_t masked(uint64_t c, uint32_t m) { return c & (uint64_t)(int64_t)(int32_t)m; }

// A run's factors e^{2 pi i (C + sum_i lam_i x_i)} (apply_run_phase) with
// the register bits LM known when the pass is compiled.  CZ (wave-uniform):
// C is zero in every lane, as it is for a run of controlled phases with no
// X frame on their qubits; then a run with one register bit multiplies only
// the registers with that bit set, and a run with none is the identity.
// (The full product multiplies the others by e^0, exactly 1, so the results
// are the same.)  The factor e^{2 pi i C} is taken in a branch of its own
// rather than beside the short form: two forms of the whole product would
// hold more registers than the tile leaves free.
template <typename R, int RB, uint32_t LM>
__device__ __forceinline__ void run_phase(cplx<R> (&v)[1 << RB], typename Turns<R>::T C,
                                          const typename Turns<R>::T (&lam)[RB], bool cz) {
    constexpr int NB = __builtin_popcount(LM);
    if constexpr (NB == 1) {
        constexpr int I = __builtin_ctz(LM);
        const cplx<R> e = expi_turns(lam[I]);
        cplx<R> w1 = e;
        if (!cz) {
            const cplx<R> w0 = expi_turns(C);
            w1 = cmul(w0, e);
            sfor<(1 << RB)>([&](auto Jc) __attribute__((always_inline)) {
                constexpr int j = decltype(Jc)::value;
                if constexpr (((j >> I) & 1) == 0) v[j] = cmul(w0, v[j]);
            });
        }
        sfor<(1 << RB)>([&](auto Jc) __attribute__((always_inline)) {
            constexpr int j = decltype(Jc)::value;
            if constexpr (((j >> I) & 1) != 0) v[j] = cmul(w1, v[j]);
        });
    } else if constexpr (NB == 0) {
        if (!cz) apply_run_phase<R, RB>(v, C, lam, LM);
    } else {
        apply_run_phase<R, RB>(v, C, lam, LM);
    }
}

// The run's register-only gates: table T (2^RB entries, index j ^ fr);
// entries whose bit in tmask is clear are exactly 1 and skipped (RB <= 5).
template <typename R, int RB>
__device__ __forceinline__ void apply_table(cplx<R> (&v)[1 << RB], kptr<cplx<R>> T, uint32_t fr, uint32_t tmask) {
    sfor<(1 << RB)>([&](auto Jc) __attribute__((always_inline)) {
        constexpr int j = decltype(Jc)::value;
        const uint32_t t = (uint32_t)j ^ fr;
        if (RB > 5 || ((tmask >> t) & 1u)) v[j] = cmul(T[t], v[j]);
    });
}

// Register bits of frame f, in register-index order (RQ: physical qubit of
// each register bit).
template <int RB>
__device__ __forceinline__ uint32_t reg_frame(uint32_t f, const uint8_t (&rq)[8]) {
    uint32_t r = 0;
#pragma unroll
    for (int i = 0; i < RB; i++) r |= ((f >> rq[i]) & 1u) << i;
    return r;
}

}  // namespace jit
}  // namespace tqs
