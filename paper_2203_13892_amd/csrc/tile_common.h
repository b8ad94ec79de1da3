// Device code shared by the pass kernels: the tile's complex type and
// arithmetic, the launch records, read-only data access, compile-time
// loops, the phase exponential, the phase-run multiply and the sampling
// partials of a tile.  Self-contained (no library headers), so that kernels
// compiled at run time for one plan include it unchanged.
#pragma once

#include "device_types.h"

namespace tqs {

constexpr uint32_t kInit = 0xFFFFFFFFu;  // src slot: start from |0..0>

template <typename R>
struct alignas(2 * sizeof(R)) cplx {
    R re, im;
};

template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

// acc + a b as four fused multiply-adds (each product term accumulates
// directly; no separate product and add)
template <typename R>
__device__ __forceinline__ cplx<R> cmac(cplx<R> acc, cplx<R> a, cplx<R> b) {
    acc.re = acc.re + a.re * b.re;
    acc.re = acc.re - a.im * b.im;
    acc.im = acc.im + a.re * b.im;
    acc.im = acc.im + a.im * b.re;
    return acc;
}

template <typename R>
__device__ __forceinline__ cplx<R> cneg_if(cplx<R> a, uint32_t neg) {
    // sign flip as an integer xor, so uniform values stay in scalar registers
    if constexpr (sizeof(R) == 4) {
        const uint32_t m = neg ? 0x80000000u : 0u;
        return {__uint_as_float(__float_as_uint(a.re) ^ m), __uint_as_float(__float_as_uint(a.im) ^ m)};
    } else {
        const unsigned long long m = neg ? 0x8000000000000000ull : 0ull;
        return {__longlong_as_double((long long)((unsigned long long)__double_as_longlong(a.re) ^ m)),
                __longlong_as_double((long long)((unsigned long long)__double_as_longlong(a.im) ^ m))};
    }
}

// Negates the real and/or imaginary part (integer sign flips).
template <typename R>
__device__ __forceinline__ cplx<R> cneg_parts(cplx<R> a, uint32_t neg_re, uint32_t neg_im) {
    if constexpr (sizeof(R) == 4) {
        return {__uint_as_float(__float_as_uint(a.re) ^ (neg_re << 31)),
                __uint_as_float(__float_as_uint(a.im) ^ (neg_im << 31))};
    } else {
        return {__longlong_as_double((long long)((unsigned long long)__double_as_longlong(a.re) ^
                                                 ((unsigned long long)neg_re << 63))),
                __longlong_as_double((long long)((unsigned long long)__double_as_longlong(a.im) ^
                                                 ((unsigned long long)neg_im << 63)))};
    }
}

// Per-node noise metadata in device memory.
struct NodeMeta {
    const uint32_t *frame0;  // [2 * node]: x, z at node start
    const uint32_t *ev_off;  // [node + 1]
    const uint32_t *ev_pos;  // (pass << 16) | position of the first op that sees it
    const uint32_t *ev_dx;
    const uint32_t *ev_dz;
    // frame tables (specialised kernels): per node ~0u, or the offset in
    // ct_dir of [count, (pass, first ctab entry) x count]: for those passes
    // the node's register-only phase tables with its own frames applied
    const uint32_t *ct_off;
    const uint32_t *ct_dir;
    const void *ctab;  // cplx<R> entries
};


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
    const uint32_t *perm;  // NULL, or the computed-state index of each launched state
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

// A compile-time integer as a type (decltype(x)::value).
template <int N>
struct IC {
    static constexpr int value = N;
};

// 0, .., N-1 as a parameter pack (the compiler's integer-sequence builtin).
template <int... Is>
struct ISeq {};
template <typename T, T... Is>
struct ISeqOf {
    using type = ISeq<Is...>;
};
template <int N>
using MakeISeq = typename __make_integer_seq<ISeqOf, int, N>::type;

// Compile-time loop: f(IC<0>{}), .., f(IC<N-1>{}) -- every register index
// stays a constant, so the tile never leaves registers.
template <typename F, int... Is>
__device__ __forceinline__ void sfor_impl(F &&f, ISeq<Is...>) {
    (f(IC<Is>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void sfor(F &&f) {
    sfor_impl(f, MakeISeq<N>{});
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

}  // namespace tqs
