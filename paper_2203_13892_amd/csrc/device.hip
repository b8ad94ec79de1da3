// Device side of tqsim for gfx950: gate-apply pass kernel, sampling
// kernels, Pauli-frame materialisation, copy probe, and the executor that
// walks the simulation tree.
//
// Noise is carried as a per-trajectory Pauli frame F = i^k X^x Z^z: the
// stored state s satisfies psi = F s.  A gate G is applied to s as
// F^dagger G F, which for a Pauli F is G with its local indices xor-ed by
// the frame's X bits and signs from its Z bits, so a noise event costs no
// memory traffic: it only updates (x, z).  At the leaf, the outcome of psi
// is the outcome of s with its index xor-ed by x.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <atomic>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>

#include "tqs_internal.h"
#include "pass_kernel.h"

namespace tqs {

// Sampling reads the state in logical index order y (bit q of y is
// logical qubit q) while the stored state s is indexed by physical
// positions: logical qubit q sits at bit lay[q], so y maps to
// P(y) = sum_q y_q 2^lay[q].  Blocks are the 2^b logical indices that share
// their high bits; their FP64 masses come from two kernels: per chunk of
// 2^c physically consecutive amplitudes (coalesced reads) the sums per
// block the chunk touches, then per block the sum over its chunks.
struct SampleMap {
    uint32_t n, b, c;   // qubits, block log, chunk log
    uint32_t kc;        // block bits among the chunk's c low positions
    uint32_t part_log;  // log2 partial sums per state: (n - c) + kc
    uint32_t cmask;     // positions of logical qubits b..n-1 (block bits)
    uint32_t smask;     // positions of logical qubits 0..b-1
    uint8_t lay[32];    // logical qubit -> physical position
    // partials written per tile by the last leaf pass instead (tiled != 0):
    // pattern bits, tile-index bits, tile-index bits inside a block, and
    // per block-index bit its source (0x80 | pattern bit, or tile bit)
    uint32_t tiled, kv, nfree, tfree;
    uint8_t bsrc[32];
};

// Sampling of one chunk of leaves of one plan (a segment of a launch).
template <typename R>
struct SampleArgs {
    const cplx<R> *states;
    uint64_t slot_amps;
    const uint32_t *slots;     // state slot per leaf of the chunk
    const uint32_t *node_ids;  // global node id per leaf of the chunk
    const uint32_t *rep;       // per leaf: index of its distinct state
    const uint32_t *rep_slots; // state slot per distinct state
    double *part, *sums;       // partial and block sums per distinct state
    const double *leaf_u;
    const uint32_t *leaf_fx;
    const uint32_t *leaf_flip;  // read-out flip mask per leaf
    uint64_t *outcomes;
    uint64_t leaf_first;       // first leaf of the run's outcome array
    uint32_t leaf_off, count;  // node id of leaf 0, leaves in the chunk
    uint32_t wg_begin[3];      // first workgroup in the partials / gather / sample launches
    uint32_t reps;             // distinct states of the chunk
    SampleMap m;
};

// One segment by value, or a table of segments sorted by wg_begin.
template <typename R>
struct SampleLaunch {
    SampleArgs<R> one;
    const SampleArgs<R> *segs;
    uint32_t nseg;  // 0: `one` is the launch
};

// The segment of workgroup `wg`, by reference into the launch argument or
// the segment table: its arrays (block map, layout) are then read in place
// (a local copy indexed by a loop variable would live in scratch memory).
template <typename R>
__device__ __forceinline__ const SampleArgs<R> &sample_seg(const SampleLaunch<R> &sl, int stage, uint32_t wg,
                                                           uint32_t *local) {
    if (sl.nseg == 0) {
        *local = wg;
        return sl.one;
    }
    const SampleArgs<R> *segs = sl.segs;
    uint32_t lo = 0, hi = sl.nseg;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (segs[mid].wg_begin[stage] <= wg) lo = mid;
        else hi = mid;
    }
    *local = wg - segs[lo].wg_begin[stage];
    return segs[lo];
}

// Partial masses: one workgroup per (state, chunk).  Thread t reads the
// chunk offsets o = t + 256 q (coalesced), so the offset's low 8 bits are the
// thread's and its high bits are q.  Each thread first adds, in registers,
// its values whose q differ only in non-block positions; the remaining
// values go to LDS at (block part of o, then the thread's non-block bits),
// and each run of threads that share a block part is summed pairwise.
template <typename R>
__global__ __launch_bounds__(kThreads) void block_partials_kernel(SampleLaunch<R> sl) {
    constexpr uint32_t kQ = 16;  // values per thread (chunk of at most 4096)
    __shared__ double buf[kThreads * kQ];
    uint32_t local;
    const SampleArgs<R> &sa = sample_seg(sl, 0, blockIdx.x, &local);
    const SampleMap &m = sa.m;
    const uint32_t nch = 1u << (m.n - m.c);
    if (local >= sa.reps * nch) return;
    const uint32_t k = local / nch, ch = local % nch;
    const cplx<R> *states = sa.states;
    const uint64_t slot_amps = sa.slot_amps;
    const uint32_t *slots = sa.rep_slots;
    double *part = sa.part;
    const uint32_t t = threadIdx.x;
    const uint32_t tb = m.c < 8 ? m.c : 8u, qb = m.c - tb;
    const uint32_t cm = m.cmask & ((1u << m.c) - 1u);
    const uint32_t cm_t = cm & ((1u << tb) - 1u), cm_q = cm >> tb;
    const uint32_t ct_bits = (uint32_t)__builtin_popcount(cm_t);
    const uint32_t st = tb - ct_bits;  // the thread's non-block bits
    uint32_t ct = 0, stt = 0;
    for (uint32_t bit = 0, nc = 0, ns = 0; bit < tb; bit++) {
        const uint32_t one = (t >> bit) & 1u;
        if ((cm_t >> bit) & 1u) ct |= one << nc++;
        else stt |= one << ns++;
    }
    const bool active = t < (1u << tb);
    const cplx<R> *s = states + (uint64_t)slots[k] * slot_amps + ((uint64_t)ch << m.c);
    // (selects, not branches, keep the 16 values in fixed registers)
    double acc[kQ];
#pragma unroll
    for (uint32_t q = 0; q < kQ; q++) {
        const bool live = active && q < (1u << qb);
        const cplx<R> v = s[live ? t + (q << tb) : 0u];
        const double a2 = (double)v.re * (double)v.re + (double)v.im * (double)v.im;
        acc[q] = live ? a2 : 0.0;
    }
#pragma unroll
    for (uint32_t b = 0; b < 4; b++) {
        const bool on = b < qb && !((cm_q >> b) & 1u);
#pragma unroll
        for (uint32_t q = 0; q < kQ; q++)
            if (!(q & (1u << b))) acc[q] += on ? acc[q | (1u << b)] : 0.0;
    }
    // values left: q with every non-block bit clear
    const uint32_t sq = ((1u << qb) - 1u) & ~cm_q;
    if (active) {
#pragma unroll
        for (uint32_t q = 0; q < kQ; q++) {
            if (q < (1u << qb) && (q & sq) == 0) {
                uint32_t cq = 0;
                for (uint32_t bit = 0, nc = 0; bit < qb; bit++)
                    if ((cm_q >> bit) & 1u) cq |= ((q >> bit) & 1u) << nc++;
                buf[((((cq << ct_bits) | ct)) << st) | stt] = acc[q];
            }
        }
    }
    __syncthreads();
    const uint32_t nvals = 1u << (m.kc + st);
    for (uint32_t h = 1; h < (1u << st); h <<= 1) {
        for (uint32_t i = t; i < (nvals >> 1) / h; i += kThreads) {
            const uint32_t e = i * 2 * h;
            buf[e] += buf[e + h];
        }
        __syncthreads();
    }
    double *out = part + ((uint64_t)k << m.part_log) + ((uint64_t)ch << m.kc);
    for (uint32_t j = t; j < (1u << m.kc); j += kThreads) out[j] = buf[j << st];
}

// Block masses in logical block order: block B's amplitudes lie in the
// chunks spelled by P(B 2^b) plus any value of the in-block positions above
// the chunk, at the same partial index in each.
template <typename R>
__global__ __launch_bounds__(kThreads) void block_gather_kernel(SampleLaunch<R> sl) {
    uint32_t local;
    const SampleArgs<R> &sa = sample_seg(sl, 1, blockIdx.x, &local);
    const SampleMap &m = sa.m;
    const uint32_t nblocks = 1u << (m.n - m.b);
    const double *part = sa.part;
    double *sums = sa.sums;
    if (m.tiled) {
        // partials per tile.  A workgroup takes RW consecutive (state, fixed
        // block bits, pattern) items, so neighbouring threads read
        // neighbouring patterns, and splits each item's tiles (those that
        // differ in in-block positions only) into 2^ls interleaved shares;
        // every share sums its tiles in increasing order, then the shares
        // are added in order (a fixed order: the result is deterministic)
        __shared__ double red[kThreads];
        const uint32_t nb = __popc(m.tfree);
        const uint32_t ls = nb < 3u ? nb : 3u;
        const uint32_t RW = kThreads >> ls;
        const uint32_t sidx = threadIdx.x / RW, ri = threadIdx.x % RW;
        const uint64_t gid = (uint64_t)local * RW + ri;
        const bool live = gid < (uint64_t)sa.reps * nblocks;
        // the share's fixed low part: sidx deposited into the lowest ls bits of tfree
        uint32_t mlo = 0, low = 0;
        for (uint32_t bits = m.tfree, i = 0; i < ls; i++) {
            const uint32_t bt = bits & (0u - bits);
            mlo |= bt;
            if ((sidx >> i) & 1u) low |= bt;
            bits ^= bt;
        }
        const uint32_t mhi = m.tfree ^ mlo;
        double acc = 0.0;
        uint32_t k = 0, B = 0;
        if (live) {
            k = (uint32_t)(gid / nblocks);
            const uint32_t r = (uint32_t)(gid % nblocks);
            const uint32_t jv = r & ((1u << m.kv) - 1u), tc = r >> m.kv;
            uint32_t tfix = 0;
            for (uint32_t i = 0, nf = 0; i < m.n - m.b; i++) {
                const uint32_t src = m.bsrc[i];
                uint32_t bit;
                if (src & 0x80u) {
                    bit = (jv >> (src & 0x7Fu)) & 1u;
                } else {
                    bit = (tc >> nf++) & 1u;
                    tfix |= bit << src;
                }
                B |= bit << i;
            }
            const double *pk = part + ((uint64_t)k << (m.nfree + m.kv)) + jv;
            const uint32_t base = tfix | low;
            const uint32_t cnt = 1u << (nb - ls);
            // four loads in flight: subsets of mhi in increasing order, dealt
            // round-robin to four accumulators
            double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
            uint32_t h = 0;
            for (uint32_t i = 0; i < cnt; i += 4) {
                const uint32_t h1 = (h - mhi) & mhi, h2 = (h1 - mhi) & mhi, h3 = (h2 - mhi) & mhi;
                a0 += pk[(uint64_t)(base | h) << m.kv];
                if (i + 1 < cnt) a1 += pk[(uint64_t)(base | h1) << m.kv];
                if (i + 2 < cnt) a2 += pk[(uint64_t)(base | h2) << m.kv];
                if (i + 3 < cnt) a3 += pk[(uint64_t)(base | h3) << m.kv];
                h = (h3 - mhi) & mhi;
            }
            acc = (a0 + a1) + (a2 + a3);
        }
        red[threadIdx.x] = acc;
        __syncthreads();
        if (live && sidx == 0) {
            double t = 0.0;
            for (uint32_t q = 0; q < (1u << ls); q++) t += red[q * RW + ri];
            sums[(uint64_t)k * nblocks + B] = t;
        }
        return;
    }
    const uint64_t gid = (uint64_t)local * kThreads + threadIdx.x;
    if (gid >= (uint64_t)sa.reps * nblocks) return;
    const uint32_t k = (uint32_t)(gid / nblocks), B = (uint32_t)(gid % nblocks);
    uint32_t pb = 0;
    for (uint32_t q = m.b; q < m.n; q++) pb |= ((B >> (q - m.b)) & 1u) << m.lay[q];
    uint32_t j = 0, nc = 0;
    for (uint32_t bit = 0; bit < m.c; bit++)
        if ((m.cmask >> bit) & 1u) {
            j |= ((pb >> bit) & 1u) << nc;
            nc++;
        }
    const uint32_t chunk0 = pb >> m.c;
    const uint32_t sh = m.smask >> m.c;
    const double *pk = part + ((uint64_t)k << m.part_log);
    double acc = 0.0;
    uint32_t sub = 0;
    do {
        acc += pk[((uint64_t)(chunk0 | sub) << m.kc) | j];
        sub = (sub - sh) & sh;  // next subset of sh, increasing
    } while (sub != 0);
    sums[gid] = acc;
}

// Inverse-CDF sampling of one leaf per workgroup, in the logical index
// order of the true state psi = F s: with the frame's X bits in logical
// order xl, psi's block B_L is s's block B_L ^ (xl >> b) and inside it
// index y is s's (y ^ xl) low bits, read at physical position P(.).  The
// outcome is min { y : sum_{y' <= y} |psi_y'|^2 > u T } with FP64 sums.
// Exclusive prefix of part[0..kThreads) into pre[], plus base, in a fixed
// order (deterministic): an inclusive scan inside each wave by shuffles,
// then the four wave totals in sequence.  Returns the total (base included)
// to every thread.  All threads call it; part[] must be written before.
__device__ __forceinline__ double block_scan(const double *part, double *pre, double base, double *wave_tot) {
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
    double x = part[tid];
#pragma unroll
    for (uint32_t d = 1; d < 64; d <<= 1) {
        const double y = __shfl_up(x, d);
        if (lane >= d) x += y;
    }
    const double ex = __shfl_up(x, 1);  // exclusive: inclusive of lane - 1
    if (lane == 63) wave_tot[wv] = x;
    __syncthreads();
    double off = base;
    for (uint32_t w = 0; w < wv; w++) off += wave_tot[w];
    pre[tid] = lane ? off + ex : off;
    double tot = base;
    for (uint32_t w = 0; w < kThreads / 64; w++) tot += wave_tot[w];
    __syncthreads();
    return tot;
}

template <typename R>
__global__ __launch_bounds__(kThreads) void sample_kernel(SampleLaunch<R> sl) {
    __shared__ double part[kThreads];
    __shared__ uint32_t ptab[3][64];  // P of the in-block index, by 6-bit digit
    __shared__ double pre[kThreads];
    __shared__ double wave_tot[kThreads / 64];
    __shared__ uint32_t hit;
    __shared__ double cum_sh;
    uint32_t k;
    const SampleArgs<R> &sa = sample_seg(sl, 2, blockIdx.x, &k);
    if (k >= sa.count) return;
    const SampleMap &m = sa.m;
    const uint32_t tid = threadIdx.x;
    const uint32_t b = m.b, nblocks = 1u << (m.n - m.b);
    const cplx<R> *states = sa.states;
    const uint64_t slot_amps = sa.slot_amps;
    const uint32_t *slots = sa.slots;
    const double *sums = sa.sums, *leaf_u = sa.leaf_u;
    const uint32_t *leaf_fx = sa.leaf_fx;
    uint64_t *outcomes = sa.outcomes;
    const uint64_t leaf_first = sa.leaf_first;
    const uint32_t lam = sa.node_ids[k] - sa.leaf_off;
    const double u = leaf_u[lam];
    const uint32_t x = leaf_fx[lam];
    const uint32_t xb = x >> b, xlow = x & ((1u << b) - 1u);
    const double *S = sums + (uint64_t)sa.rep[k] * nblocks;
    const cplx<R> *psi = states + (uint64_t)slots[k] * slot_amps;
    if (tid < 192) {
        const uint32_t h = tid >> 6;
        const uint32_t v = (tid & 63u) << (6 * h);
        uint32_t pv = 0;
        for (uint32_t q = 0; q < b; q++) pv |= ((v >> q) & 1u) << m.lay[q];
        ptab[h][tid & 63u] = pv;
    }
    auto plow = [&](uint32_t v) { return ptab[0][v & 63u] | ptab[1][(v >> 6) & 63u] | ptab[2][(v >> 12) & 63u]; };

    // logical block prefix: thread t owns blocks [t*seg, (t+1)*seg)
    const uint32_t seg = (nblocks + kThreads - 1) / kThreads;
    const uint32_t b0 = tid * seg, b1 = min(nblocks, b0 + seg);
    double s = 0.0;
    for (uint32_t B = b0; B < b1; B++) s += S[B ^ xb];
    part[tid] = s;
    if (tid == 0) hit = 0xFFFFFFFFu;
    __syncthreads();
    const double t = u * block_scan(part, pre, 0.0, wave_tot);
    {
        double run = pre[tid];
        for (uint32_t B = b0; B < b1; B++) {
            run += S[B ^ xb];
            if (run > t) {
                atomicMin(&hit, B);
                break;
            }
        }
    }
    __syncthreads();
    uint32_t BL = hit;
    __syncthreads();  // every thread has read `hit` before thread 0 rewrites it
    if (BL == 0xFFFFFFFFu) {
        // rounding left no crossing: last block with nonzero mass
        if (tid == 0) {
            uint32_t last = 0;
            for (uint32_t B = 0; B < nblocks; B++)
                if (S[B ^ xb] > 0.0) last = B;
            hit = last;
        }
        __syncthreads();
        BL = hit;
        __syncthreads();
    }
    // cumulative mass before block BL (same order as above)
    if (tid == 0) {
        const uint32_t owner = BL / seg;
        double run = pre[owner];
        for (uint32_t B = owner * seg; B < BL; B++) run += S[B ^ xb];
        cum_sh = run;
        hit = 0xFFFFFFFFu;
    }
    __syncthreads();
    const uint32_t Bp = BL ^ xb;
    uint32_t pB = 0;
    for (uint32_t q = b; q < m.n; q++) pB |= ((Bp >> (q - b)) & 1u) << m.lay[q];
    const cplx<R> *blk = psi + pB;
    const uint32_t nb = 1u << b;
    const uint32_t iseg = (nb + kThreads - 1) / kThreads;
    const uint32_t y0 = tid * iseg, y1 = min(nb, y0 + iseg);
    // (blocks of up to 16 values per thread are read once and kept)
    constexpr uint32_t kKeep = 16;
    const bool keep = iseg <= kKeep;
    double pv[kKeep];
    s = 0.0;
    if (keep) {
#pragma unroll
        for (uint32_t i = 0; i < kKeep; i++) {
            const uint32_t y = y0 + i;
            double a2 = 0.0;
            if (y < y1) {
                const cplx<R> v = blk[plow(y ^ xlow)];
                a2 = (double)v.re * (double)v.re + (double)v.im * (double)v.im;
            }
            pv[i] = a2;
            s += a2;
        }
    } else {
        for (uint32_t y = y0; y < y1; y++) {
            const cplx<R> v = blk[plow(y ^ xlow)];
            s += (double)v.re * (double)v.re + (double)v.im * (double)v.im;
        }
    }
    part[tid] = s;
    __syncthreads();
    block_scan(part, pre, cum_sh, wave_tot);
    {
        double run = pre[tid];
        if (keep) {
            bool found = false;
#pragma unroll
            for (uint32_t i = 0; i < kKeep; i++) {
                run += pv[i];
                if (!found && y0 + i < y1 && run > t) {
                    atomicMin(&hit, y0 + i);
                    found = true;
                }
            }
        } else {
            for (uint32_t y = y0; y < y1; y++) {
                const cplx<R> v = blk[plow(y ^ xlow)];
                run += (double)v.re * (double)v.re + (double)v.im * (double)v.im;
                if (run > t) {
                    atomicMin(&hit, y);
                    break;
                }
            }
        }
    }
    __syncthreads();
    if (tid == 0) {
        uint32_t y = hit;
        if (y == 0xFFFFFFFFu) {
            y = 0;
            for (uint32_t i = 0; i < nb; i++) {
                const cplx<R> v = blk[plow(i ^ xlow)];
                if ((double)v.re * v.re + (double)v.im * v.im > 0.0) y = i;
            }
        }
        // read-out channel: measured bits flip after the measurement
        outcomes[lam - leaf_first] = (((uint64_t)BL << b) | y) ^ sa.leaf_flip[lam];
    }
}

// Standalone Pauli application in logical order: out(y) = i^k (-1)^{z.w}
// in(w) with w = P(y) ^ x, i.e. the frame F = i^k X^x Z^z applied to a
// stored state, read out with logical qubit q at bit q.
template <typename R>
__global__ __launch_bounds__(kThreads) void frame_apply_kernel(const cplx<R> *in, cplx<R> *out,
                                                               uint64_t amps, uint32_t x, uint32_t z,
                                                               uint32_t k, SampleMap m) {
    const uint64_t y = (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (y >= amps) return;
    uint32_t py = 0;
    for (uint32_t q = 0; q < m.n; q++) py |= (((uint32_t)y >> q) & 1u) << m.lay[q];
    const uint32_t w = py ^ x;
    cplx<R> v = in[w];
    v = cneg_if(v, __builtin_popcount(z & w) & 1u);
    for (uint32_t i = 0; i < (k & 3u); i++) v = cplx<R>{-v.im, v.re};
    out[y] = v;
}

// Streaming copy (bandwidth probe): 16-byte loads and stores.
__global__ __launch_bounds__(kThreads) void copy_kernel(const uint4 *__restrict__ in,
                                                        uint4 *__restrict__ out, uint64_t n16) {
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    for (uint64_t i = (uint64_t)blockIdx.x * kThreads + threadIdx.x; i < n16; i += stride)
        out[i] = in[i];
}

// ------------------------------------------------------------- executor --

static tqs_status hip_fail(hipError_t e, const char *what) {
    return fail(TQS_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                      \
    do {                                         \
        hipError_t _e = (expr);                  \
        if (_e != hipSuccess) return hip_fail(_e, what); \
    } while (0)

static inline uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

struct Frame {
    uint32_t x = 0, z = 0, k = 0;  // i^k X^x Z^z
};

// E * F for Pauli E = i^ke X^ex Z^ez:  X^ex Z^ez X^fx Z^fz = (-1)^{ez.fx} X^(ex^fx) Z^(ez^fz)
static inline Frame compose(uint32_t ex, uint32_t ez, uint32_t ke, const Frame &f) {
    Frame r;
    r.x = ex ^ f.x;
    r.z = ez ^ f.z;
    r.k = (ke + f.k + 2u * ((uint32_t)__builtin_popcount(ez & f.x) & 1u)) & 3u;
    return r;
}

struct Layout {
    uint64_t amp_bytes, state_bytes;
    uint32_t slots_total;
    std::vector<uint32_t> slot_base;  // per level
    uint32_t scratch_slot;
    uint64_t off_states;  // first state slot
    uint64_t off_meta, off_mats, off_ops, off_passes, off_terms, off_dgates, off_frame0, off_evoff,
        off_evpos, off_evdx, off_evdz, off_leafu, off_leaffx, off_flip, off_sched, off_ctoff, off_ctab, off_sums,
        off_part, off_out, total;
    uint64_t n_sched;
};

// Offsets are absolute in the workspace: states from `states_at`, the
// metadata and sampling regions from `meta_at` (by default right after the
// states).  `total` is the end of the metadata regions.
static Layout make_layout(const tqs_plan *p, uint64_t n_events, uint64_t n_leaves_out, uint64_t n_sched,
                          uint64_t states_at = 0, uint64_t meta_at = ~0ull, uint64_t n_ctab = 0) {
    Layout L;
    L.off_states = states_at;
    L.amp_bytes = p->prec == TQS_C64 ? 8 : 16;
    L.state_bytes = L.amp_bytes << p->n;
    uint32_t s = 0;
    for (size_t l = 0; l < p->chunk.size(); l++) {
        L.slot_base.push_back(s);
        s += p->chunk[l];
    }
    L.scratch_slot = s;
    L.slots_total = s + 1;
    uint64_t o = meta_at != ~0ull ? meta_at : align256(states_at + (uint64_t)L.slots_total * L.state_bytes);
    L.off_meta = o;
    L.off_mats = o;
    o = align256(o + p->mats.size() * L.amp_bytes);
    L.off_ops = o;
    o = align256(o + p->ops.size() * sizeof(OpDesc));
    L.off_passes = o;
    o = align256(o + p->passes.size() * sizeof(PassDesc));
    L.off_terms = o;
    o = align256(o + p->terms.size() * sizeof(DiagTerm));
    L.off_dgates = o;
    o = align256(o + p->dgates.size() * sizeof(DiagGate));
    L.off_frame0 = o;
    o = align256(o + p->n_nodes * 8);
    L.off_evoff = o;
    o = align256(o + (p->n_nodes + 1) * 4);
    L.off_evpos = o;
    o = align256(o + n_events * 4);
    L.off_evdx = o;
    o = align256(o + n_events * 4);
    L.off_evdz = o;
    o = align256(o + n_events * 4);
    L.off_leafu = o;
    o = align256(o + p->n_leaves * 8);
    L.off_leaffx = o;
    o = align256(o + p->n_leaves * 4);
    L.off_flip = o;
    o = align256(o + p->n_leaves * 4);
    L.off_sched = o;
    L.n_sched = n_sched;
    o = align256(o + n_sched * 4);
    L.off_ctoff = o;
    o = align256(o + p->n_nodes * 4);
    L.off_ctab = o;
    o = align256(o + n_ctab * L.amp_bytes);
    L.off_sums = o;
    const uint64_t nblocks = 1ull << (p->n - p->sample_b);
    o = align256(o + (uint64_t)p->chunk.back() * nblocks * 8);
    L.off_part = o;
    o = align256(o + std::max((uint64_t)p->chunk.back() << p->part_log,
                              (uint64_t)p->chunk.back() << (p->samp_nfree + p->samp_kv)) * 8);
    L.off_out = o;
    o = align256(o + n_leaves_out * 8);
    L.total = o;
    return L;
}

// Chunk task of the depth-first walk: `count` consecutive nodes of `level`
// starting at local index `first`.  Of those, `ccount` distinct states are
// computed; a node whose parent state, starting frame and event list equal an
// earlier node's of the chunk shares that node's state (Sec. 6, inter-shot
// redundancy).  Tables at `sched` (u32): per node its id, state slot and the
// index of the computed state it uses; then per computed state its node id,
// source slot and destination slot.
struct Task {
    uint32_t level;
    uint64_t first;
    uint32_t count, ccount;
    uint64_t sched;
    uint64_t node_ids() const { return sched; }
    uint64_t slot_of() const { return sched + count; }
    uint64_t rep_of() const { return sched + 2ull * count; }
    uint64_t cnode() const { return sched + 3ull * count; }
    uint64_t csrc() const { return cnode() + ccount; }
    uint64_t cdst() const { return cnode() + 2ull * ccount; }
};

struct HostMeta;
static bool same_history(const HostMeta &hm, uint32_t a, uint32_t b);
static uint64_t history_hash(const HostMeta &hm, uint32_t a);

// History keys of a chunk's computed states: open addressing with linear
// probing, at most half full (a chunk computes at most `chunk` states).
// Equal keys may belong to different histories, so a lookup visits every
// entry with its key.
struct SeenTable {
    std::vector<uint64_t> key;
    std::vector<uint32_t> val;  // computed index; kEmpty marks a free entry
    uint64_t mask = 0;
    static constexpr uint32_t kEmpty = 0xFFFFFFFFu;
    void reset(uint64_t n) {
        uint64_t cap = 16;
        while (cap < 2 * n) cap <<= 1;
        if (key.size() != cap) {
            key.assign(cap, 0);
            val.assign(cap, kEmpty);
        } else {
            std::fill(val.begin(), val.end(), kEmpty);
        }
        mask = cap - 1;
    }
    uint64_t home(uint64_t k) const { return (k ^ (k >> 29)) & mask; }
    template <typename F>
    int64_t find(uint64_t k, F &&match) const {
        for (uint64_t i = home(k); val[i] != kEmpty; i = (i + 1) & mask)
            if (key[i] == k && match(val[i])) return val[i];
        return -1;
    }
    void insert(uint64_t k, uint32_t v) {
        uint64_t i = home(k);
        while (val[i] != kEmpty) i = (i + 1) & mask;
        key[i] = k;
        val[i] = v;
    }
};

// Depth-first chunk walk of the subtrees [first0, last0).  hm == NULL
// computes every node.
static void build_schedule(const tqs_plan *p, uint64_t first0, uint64_t last0, std::vector<Task> *tasks,
                           std::vector<uint32_t> *sched, const std::vector<uint32_t> &slot_base,
                           const HostMeta *hm) {
    const uint32_t L = (uint32_t)p->arity.size();
    struct Frame_ {
        uint32_t level;
        uint64_t p0, p1;                 // parent range at level-1 (for level 0: subtree range)
        uint64_t next;                   // next child to process (local index at `level`)
        std::vector<uint32_t> pslot;     // state slot of each parent in [p0, p1)
    };
    std::vector<Frame_> st;
    st.push_back({0, first0, last0, first0, {}});
    std::vector<uint32_t> slot, rep, cnode, csrc;
    SeenTable seen;  // history key -> computed index
    while (!st.empty()) {
        Frame_ &f = st.back();
        const uint32_t l = f.level;
        const uint64_t A = p->arity[l];
        const uint64_t c_end = l == 0 ? f.p1 : f.p1 * A;
        if (f.next >= c_end) {
            st.pop_back();
            continue;
        }
        // the chunk takes nodes until its computed states fill the level's
        // slots; nodes that share an earlier node's state take no slot
        const uint64_t c0 = f.next;
        slot.clear();
        rep.clear();
        cnode.clear();
        csrc.clear();
        if (hm) seen.reset(p->chunk[l]);
        uint64_t c = c0;
        for (; c < c_end; c++) {
            const uint32_t node = (uint32_t)(p->level_offset[l] + c);
            const uint32_t from = l == 0 ? kInit : f.pslot[c / A - f.p0];
            int64_t hit = -1;
            uint64_t key = 0;
            if (hm) {
                key = history_hash(*hm, node) * 0x9E3779B97F4A7C15ull + from;
                hit = seen.find(key, [&](uint32_t j) { return csrc[j] == from && same_history(*hm, cnode[j], node); });
            }
            if (hit < 0) {
                if (cnode.size() == p->chunk[l]) break;
                hit = (int64_t)cnode.size();
                cnode.push_back(node);
                csrc.push_back(from);
                if (hm) seen.insert(key, (uint32_t)hit);
            }
            rep.push_back((uint32_t)hit);
            slot.push_back(slot_base[l] + (uint32_t)hit);
        }
        const uint64_t c1 = c;
        f.next = c1;
        const uint32_t cnt = (uint32_t)(c1 - c0);
        Task t;
        t.level = l;
        t.first = c0;
        t.count = cnt;
        t.ccount = (uint32_t)cnode.size();
        t.sched = sched->size();
        for (uint64_t cc = c0; cc < c1; cc++) sched->push_back((uint32_t)(p->level_offset[l] + cc));
        sched->insert(sched->end(), slot.begin(), slot.end());
        sched->insert(sched->end(), rep.begin(), rep.end());
        sched->insert(sched->end(), cnode.begin(), cnode.end());
        sched->insert(sched->end(), csrc.begin(), csrc.end());
        for (uint32_t j = 0; j < t.ccount; j++) sched->push_back(slot_base[l] + j);
        tasks->push_back(t);
        if (l + 1 < L) st.push_back({l + 1, c0, c1, c0 * p->arity[l + 1], slot});
    }
}

struct HostMeta {
    std::vector<uint32_t> frame0;  // 2 per node
    std::vector<uint32_t> ev_off, ev_pos, ev_dx, ev_dz;
    // per node: how many of its (position-sorted) events the passes apply
    // before some op; the rest come after the level's last op and change
    // only the frame the node ends with, not its state
    std::vector<uint32_t> ev_eff;
    std::vector<uint32_t> leaf_fx;
    std::vector<Frame> leaf_frame;
};

// Two nodes compute the same state from the same parent state when they
// start from the same frame and meet the same events at the same places
// before the level's last op (later events change only their end frames).
static bool same_history(const HostMeta &hm, uint32_t a, uint32_t b) {
    if (hm.frame0[2 * a] != hm.frame0[2 * b] || hm.frame0[2 * a + 1] != hm.frame0[2 * b + 1]) return false;
    const uint32_t na = hm.ev_eff[a], nb = hm.ev_eff[b];
    if (na != nb) return false;
    for (uint32_t i = 0; i < na; i++) {
        const uint32_t ea = hm.ev_off[a] + i, eb = hm.ev_off[b] + i;
        if (hm.ev_pos[ea] != hm.ev_pos[eb] || hm.ev_dx[ea] != hm.ev_dx[eb] || hm.ev_dz[ea] != hm.ev_dz[eb])
            return false;
    }
    return true;
}

static uint64_t history_hash(const HostMeta &hm, uint32_t a) {
    uint64_t h = ((uint64_t)hm.frame0[2 * a] << 32) ^ hm.frame0[2 * a + 1];
    for (uint32_t e = hm.ev_off[a]; e < hm.ev_off[a] + hm.ev_eff[a]; e++) {
        h = (h ^ hm.ev_pos[e]) * 0x100000001B3ull;
        h = (h ^ ((uint64_t)hm.ev_dx[e] << 32 | hm.ev_dz[e])) * 0x100000001B3ull;
    }
    return h;
}

// Map the insertion list onto pass positions and Pauli masks, and compose
// each node's frame from its parent's (Sec. 3.1: a child continues from a
// copy of its parent's state, noise included).
static uint32_t to_logical(const tqs_plan *p, uint32_t x);

static void build_meta(const tqs_plan *p, const tqs_noise *nz, HostMeta *hm) {
    const uint64_t N = p->n_nodes;
    hm->frame0.assign(2 * N, 0);
    hm->ev_off.assign(N + 1, 0);
    const uint64_t E = nz->ev_gate.size();
    hm->ev_pos.resize(E);
    hm->ev_dx.resize(E);
    hm->ev_dz.resize(E);
    hm->leaf_fx.assign(p->n_leaves, 0);
    hm->leaf_frame.assign(p->n_leaves, Frame());
    hm->ev_eff.assign(N, 0);
    std::vector<Frame> fend(N);
    std::vector<std::pair<uint32_t, uint64_t>> ord;
    const uint32_t L = (uint32_t)p->arity.size();
    for (uint32_t l = 0; l < L; l++) {
        const uint64_t I = p->level_nodes[l], off = p->level_offset[l];
        // the last position at which a pass of this level applies an event
        // before an op: before a dense op at its first slot, inside a phase
        // run up to its last gate (events after it touch no op of the level)
        int64_t limit = -1;
        const tqs::Level &lv = p->levels[l];
        for (uint32_t pi = lv.pass_begin; pi < lv.pass_begin + lv.pass_count; pi++) {
            const PassDesc &pd = p->passes[pi];
            for (uint32_t oi = pd.op_begin; oi < pd.op_begin + pd.op_count; oi++) {
                const OpDesc &o = p->ops[oi];
                const uint32_t last = o.slot1 > o.slot0 ? (uint32_t)o.slot1 - 1u : (uint32_t)o.slot0;
                limit = std::max<int64_t>(limit, (int64_t)((pi << 16) | std::max<uint32_t>(o.slot0, last)));
            }
        }
        for (uint64_t m = 0; m < I; m++) {
            const uint64_t nu = off + m;
            Frame f;
            if (l > 0) f = fend[p->level_offset[l - 1] + m / p->arity[l]];
            hm->frame0[2 * nu] = f.x;
            hm->frame0[2 * nu + 1] = f.z;
            // the node's events in the order the passes meet them (gates that
            // share no qubit may run out of circuit order)
            const uint64_t e0 = nz->node_off[nu], e1 = nz->node_off[nu + 1];
            ord.clear();
            for (uint64_t e = e0; e < e1; e++) {
                const uint32_t g = nz->ev_gate[e];
                ord.push_back({(p->gate_pass[g] << 16) | p->gate_pos[g], e});
            }
            if (ord.size() <= 32) {
                // a node carries a handful of events: a stable insertion sort
                // (no scratch allocation per node)
                for (size_t i = 1; i < ord.size(); i++) {
                    const std::pair<uint32_t, uint64_t> x = ord[i];
                    size_t j = i;
                    for (; j > 0 && ord[j - 1].first > x.first; j--) ord[j] = ord[j - 1];
                    ord[j] = x;
                }
            } else {
                std::stable_sort(ord.begin(), ord.end(),
                                 [](const std::pair<uint32_t, uint64_t> &a, const std::pair<uint32_t, uint64_t> &b) {
                                     return a.first < b.first;
                                 });
            }
            for (uint64_t i = 0; i < ord.size(); i++) {
                const uint64_t e = ord[i].second, o = e0 + i;
                const uint32_t g = nz->ev_gate[e];
                const uint32_t code = nz->ev_code[e];
                uint32_t dx = 0, dz = 0, ky = 0;
                const uint32_t q[2] = {p->gate_q0[g], p->gate_q1[g]};
                for (uint32_t j = 0; j < p->gate_a[g]; j++) {
                    const uint32_t cj = (code >> (2 * j)) & 3u;
                    if (cj == 1 || cj == 2) dx |= 1u << q[j];
                    if (cj == 3 || cj == 2) dz |= 1u << q[j];
                    if (cj == 2) ky++;  // Y = i X Z
                }
                // the product of the one-qubit factors: X^dx Z^dz up to i^ky
                hm->ev_pos[o] = ord[i].first;
                hm->ev_dx[o] = dx;
                hm->ev_dz[o] = dz;
                f = compose(dx, dz, ky, f);
            }
            hm->ev_off[nu + 1] = (uint32_t)nz->node_off[nu + 1];
            uint32_t eff = 0;
            while (eff < ord.size() && (int64_t)ord[eff].first <= limit) eff++;
            hm->ev_eff[nu] = eff;
            fend[nu] = f;
            if (l == L - 1) {
                hm->leaf_fx[m] = to_logical(p, f.x);
                hm->leaf_frame[m] = f;
            }
        }
    }
}

template <typename R>
static PassArgs<R> pass_args(const tqs_plan *p, const Layout &Ly, unsigned char *ws, const Task &t,
                             uint32_t pass_idx, bool first) {
    const PassDesc &pd = p->passes[pass_idx];
    PassArgs<R> a;
    a.states = reinterpret_cast<cplx<R> *>(ws + Ly.off_states);
    a.slot_amps = 1ull << p->n;
    const uint32_t *sched = reinterpret_cast<const uint32_t *>(ws + Ly.off_sched);
    a.node_ids = sched + t.cnode();
    a.src_slot = sched + (first ? t.csrc() : t.cdst());
    a.dst_slot = sched + t.cdst();
    a.perm = nullptr;
    a.count = t.ccount;
    a.work = t.ccount * (1u << pd.nfree);
    a.pass_key = pass_idx << 16;
    a.wg_begin = 0;
    a.pass = reinterpret_cast<const PassDesc *>(ws + Ly.off_passes) + pass_idx;
    a.ops = reinterpret_cast<const OpDesc *>(ws + Ly.off_ops);
    a.mats = reinterpret_cast<const cplx<R> *>(ws + Ly.off_mats);
    a.meta.frame0 = reinterpret_cast<const uint32_t *>(ws + Ly.off_frame0);
    a.meta.ev_off = reinterpret_cast<const uint32_t *>(ws + Ly.off_evoff);
    a.meta.ev_pos = reinterpret_cast<const uint32_t *>(ws + Ly.off_evpos);
    a.meta.ev_dx = reinterpret_cast<const uint32_t *>(ws + Ly.off_evdx);
    a.meta.ev_dz = reinterpret_cast<const uint32_t *>(ws + Ly.off_evdz);
    a.meta.ct_off = reinterpret_cast<const uint32_t *>(ws + Ly.off_ctoff);
    a.meta.ct_dir = reinterpret_cast<const uint32_t *>(ws + Ly.off_sched);
    a.meta.ctab = ws + Ly.off_ctab;
    a.terms = reinterpret_cast<const DiagTerm *>(ws + Ly.off_terms);
    a.dgates = reinterpret_cast<const DiagGate *>(ws + Ly.off_dgates);
    // the last pass of the leaf level writes the sampling partials
    const tqs::Level &ll = p->levels.back();
    a.part = nullptr;
    a.psum = 0;
    a.pad = 0;
    if (p->samp_tiled && t.level + 1 == p->levels.size() && pass_idx + 1 == ll.pass_begin + ll.pass_count) {
        a.part = reinterpret_cast<double *>(ws + Ly.off_part);
        a.psum = p->samp_psum;
    }
    return a;
}

// One wave per workgroup; the register-qubit count is a compile-time tile
// width, D2 the variant with 4x4 ops.
template <typename R>
static void launch_pass_kernel(uint32_t reg_bits, bool d2, const PassLaunch<R> &pl, hipStream_t s) {
    const uint32_t grid = (pl.total + 7u) & ~7u;
#define TQS_LAUNCH(RB)                                                                          \
    do {                                                                                         \
        if (d2) hipLaunchKernelGGL((pass_kernel<R, RB, true>), dim3(grid), dim3(64), 0, s, pl);  \
        else hipLaunchKernelGGL((pass_kernel<R, RB, false>), dim3(grid), dim3(64), 0, s, pl);    \
    } while (0)
    if constexpr (sizeof(R) == 4) {
        switch (reg_bits) {
            case 4: TQS_LAUNCH(4); break;
            case 5: TQS_LAUNCH(5); break;
            default: TQS_LAUNCH(6); break;
        }
    } else {
        switch (reg_bits) {
            case 4: TQS_LAUNCH(4); break;
            default: TQS_LAUNCH(5); break;
        }
    }
#undef TQS_LAUNCH
}

// All passes of one level in one launch with the state in LDS (complex64
// tiles of four or five register qubits: two waves per SIMD leave each
// lane 256 registers, enough for the tile without spills).
static void launch_level_kernel(uint32_t reg_bits, bool d2, const LevelLaunch<float> &ll, uint32_t waves,
                                uint32_t lds_bytes, hipStream_t s) {
    const uint32_t grid = (ll.a.count + 7u) & ~7u;
    const dim3 g(grid), b(64 * waves);
    if (reg_bits == 4) {
        if (d2) hipLaunchKernelGGL((level_kernel<float, 4, true>), g, b, lds_bytes, s, ll);
        else hipLaunchKernelGGL((level_kernel<float, 4, false>), g, b, lds_bytes, s, ll);
    } else {
        if (d2) hipLaunchKernelGGL((level_kernel<float, 5, true>), g, b, lds_bytes, s, ll);
        else hipLaunchKernelGGL((level_kernel<float, 5, false>), g, b, lds_bytes, s, ll);
    }
}

constexpr int kMaxDevices = 64;

// LDS bytes one workgroup may hold on the current device (cached per device).
static uint32_t device_lds_limit() {
    static std::atomic<int> cached[kMaxDevices];  // 0: not asked yet, -1: unknown
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 0;
    int c = cached[dev].load(std::memory_order_relaxed);
    if (!c) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
            v = -1;
        cached[dev].store(v, std::memory_order_relaxed);
        c = v;
    }
    return c > 0 ? (uint32_t)c : 0u;
}

// Waves per workgroup and LDS bytes of the level kernel for level l of the
// plan, or {0, 0} when the level runs pass by pass: the generic kernels,
// complex64 tiles of at most five register qubits, two or more passes, the
// state within LDS and at most eight tiles.
struct LevelShape {
    uint32_t waves = 0, lds = 0;
};
static LevelShape level_shape(const tqs_plan *p, uint32_t l) {
    LevelShape ls;
    const tqs::Level &lv = p->levels[l];
    if (p->tune.lds_levels != 1 || p->tune.jit == 1 || lv.pass_count < 2) return ls;
    if (p->prec != TQS_C64 || p->reg_bits > 5) return ls;
    const uint64_t bytes = 8ull << p->n;
    uint32_t nfree = 0;
    for (uint32_t k = 0; k < lv.pass_count; k++) nfree = std::max<uint32_t>(nfree, p->passes[lv.pass_begin + k].nfree);
    if (nfree > 3 || bytes > device_lds_limit()) return ls;
    ls.waves = 1u << nfree;
    ls.lds = (uint32_t)bytes;
    return ls;
}

// Which kernel takes each computed state of a chunk task's pass: the
// plan-specialised kernel (when the plan has one for the pass) takes the
// states it supports, the generic kernel the rest.  perm: offset in the
// schedule of the task's computed-state indices, specialised ones first
// (kNoPerm: all states go to one kernel, in order).
struct Route {
    static constexpr uint64_t kNoPerm = ~0ull;
    uint64_t perm = kNoPerm;
    uint32_t n_jit = 0;  // states for the specialised kernel
};

// Frame tables of the computed states that need them, and where each
// node's directory starts (ct_off; ~0u: none).
struct FrameTables {
    std::vector<cd> tab;
    std::vector<uint32_t> ct_off;
};

// Routes of every (task, pass of its level), appending index lists and the
// frame-table directories to sched.
static void route_passes(const tqs_plan *p, const HostMeta &hm, const std::vector<Task> &tasks,
                         std::vector<uint32_t> *sched, std::vector<std::vector<Route>> *routes, FrameTables *ft,
                         bool jit = true) {
    routes->assign(tasks.size(), {});
    for (size_t ti = 0; ti < tasks.size(); ti++) (*routes)[ti].assign(p->levels[tasks[ti].level].pass_count, Route());
    ft->tab.clear();
    ft->ct_off.assign(p->n_nodes, 0xFFFFFFFFu);
    if (p->tune.jit != 1 || !jit) return;
    std::vector<std::vector<JitRun>> runs;
    std::vector<std::vector<JitBlock>> blks;
    jit_runs(p, &runs, &blks);
    std::vector<uint32_t> yes, no;
    // per node with frame tables: (pass, first entry) pairs
    std::vector<std::pair<uint32_t, std::vector<std::pair<uint32_t, uint32_t>>>> dirs;
    std::unordered_map<uint32_t, size_t> dir_of;
    for (size_t ti = 0; ti < tasks.size(); ti++) {
        const Task &t = tasks[ti];
        const tqs::Level &lv = p->levels[t.level];
        for (uint32_t k = 0; k < lv.pass_count; k++) {
            const uint32_t pi = lv.pass_begin + k;
            Route &r = (*routes)[ti][k];
            if (!jit_pass_supported(p, pi)) continue;
            yes.clear();
            no.clear();
            for (uint32_t c = 0; c < t.ccount; c++) {
                const uint32_t node = (*sched)[t.cnode() + c];
                const uint32_t e0 = hm.ev_off[node], e1 = hm.ev_off[node + 1];
                // only the node's events inside this pass matter for the fit
                const uint32_t *ps = hm.ev_pos.data();
                const uint32_t *pa = std::lower_bound(ps + e0, ps + e1, pi << 16);
                const uint32_t *pb = std::lower_bound(pa, ps + e1, (pi + 1) << 16);
                const JitFit fit = pa == pb ? JIT_YES
                                            : jit_fit(runs[pi], blks[pi], pi, pa, hm.ev_dx.data() + (pa - ps),
                                                      (uint32_t)(pb - pa));
                if (fit == JIT_NO) {
                    no.push_back(c);
                    continue;
                }
                yes.push_back(c);
                if (fit == JIT_TABLES) {
                    const uint32_t first = (uint32_t)ft->tab.size();
                    jit_frame_tables(p, pi, hm.frame0[2 * node], hm.ev_pos.data() + e0, hm.ev_dx.data() + e0,
                                     e1 - e0, &ft->tab);
                    auto it = dir_of.find(node);
                    if (it == dir_of.end()) {
                        it = dir_of.emplace(node, dirs.size()).first;
                        dirs.push_back({node, {}});
                    }
                    dirs[it->second].second.push_back({pi, first});
                }
            }
            r.n_jit = (uint32_t)yes.size();
            if (no.empty() || yes.empty()) continue;
            r.perm = sched->size();
            sched->insert(sched->end(), yes.begin(), yes.end());
            sched->insert(sched->end(), no.begin(), no.end());
        }
    }
    for (const auto &d : dirs) {
        ft->ct_off[d.first] = (uint32_t)sched->size();
        sched->push_back((uint32_t)d.second.size());
        for (const auto &e : d.second) {
            sched->push_back(e.first);
            sched->push_back(e.second);
        }
    }
}

// Frame-table entries route_passes may create at most.
static uint64_t table_bound(const tqs_plan *p) {
    uint64_t b = 0;
    if (p->tune.jit == 1)
        for (size_t l = 0; l < p->levels.size(); l++)
            for (uint32_t k = 0; k < p->levels[l].pass_count; k++)
                b += p->level_nodes[l] * (uint64_t)jit_table_entries(p, p->levels[l].pass_begin + k);
    return b;
}

// Schedule entries route_passes may append at most.
static uint64_t route_bound(const tqs_plan *p) {
    uint64_t b = 0;
    if (p->tune.jit == 1)
        for (size_t l = 0; l < p->levels.size(); l++)
            b += p->level_nodes[l] * (uint64_t)(p->levels[l].pass_count + 1 + 2 * p->levels[l].pass_count);
    return b;
}

template <typename R>
static hipError_t launch_jit(const tqs_plan *p, uint32_t pass_idx, PassLaunch<R> &pl, hipStream_t s) {
    const uint32_t grid = (pl.total + 7u) & ~7u;
    void *args[] = {&pl};
    return hipModuleLaunchKernel((hipFunction_t)p->jit_fn[pass_idx], grid, 1, 1, 64, 1, 1, 0, s, args, nullptr);
}

// One pass over a task's computed states, split between the kernels as
// routed.  Returns the states the specialised kernel took.
template <typename R>
static uint32_t launch_routed(const tqs_plan *p, const Layout &Ly, unsigned char *ws, hipStream_t s,
                              const Task &t, uint32_t pass_idx, bool first, const Route &r,
                              uint32_t *launches, hipError_t *err, hipEvent_t ej0, hipEvent_t ej1) {
    const bool have_jit = p->tune.jit == 1 && pass_idx < p->jit_fn.size() && p->jit_fn[pass_idx];
    const uint32_t n_jit = have_jit ? r.n_jit : 0u;
    PassLaunch<R> pl;
    std::memset(&pl, 0, sizeof pl);
    pl.one = pass_args<R>(p, Ly, ws, t, pass_idx, first);
    pl.nseg = 0;
    const uint32_t tiles = 1u << p->passes[pass_idx].nfree;
    const uint32_t *sched = reinterpret_cast<const uint32_t *>(ws + Ly.off_sched);
    *launches = 0;
    if (n_jit) {
        PassLaunch<R> pj = pl;
        if (r.perm != Route::kNoPerm) pj.one.perm = sched + r.perm;
        pj.one.count = n_jit;
        pj.one.work = n_jit * tiles;
        pj.total = pj.one.work;
        hipError_t e = ej0 ? hipEventRecord(ej0, s) : hipSuccess;
        if (e == hipSuccess) e = launch_jit<R>(p, pass_idx, pj, s);
        if (e == hipSuccess && ej1) e = hipEventRecord(ej1, s);
        *err = e;
        (*launches)++;
        if (e != hipSuccess) return n_jit;
    }
    if (n_jit < t.ccount) {
        if (n_jit) pl.one.perm = sched + r.perm + n_jit;
        pl.one.count = t.ccount - n_jit;
        pl.one.work = pl.one.count * tiles;
        pl.total = pl.one.work;
        launch_pass_kernel<R>(p->reg_bits, p->passes[pass_idx].has_d2 != 0, pl, s);
        (*launches)++;
    }
    return n_jit;
}

template <typename R>
static void launch_pass(const tqs_plan *p, const Layout &Ly, unsigned char *ws, hipStream_t s,
                        const Task &t, uint32_t pass_idx, bool first) {
    PassLaunch<R> pl;
    std::memset(&pl, 0, sizeof pl);
    pl.one = pass_args<R>(p, Ly, ws, t, pass_idx, first);
    pl.nseg = 0;
    pl.total = pl.one.work;
    launch_pass_kernel<R>(p->reg_bits, p->passes[pass_idx].has_d2 != 0, pl, s);
}

static SampleMap sample_map(const tqs_plan *p) {
    SampleMap m;
    std::memset(&m, 0, sizeof m);
    m.n = p->n;
    m.b = p->sample_b;
    m.c = std::min<uint32_t>(p->n, 12u);
    for (uint32_t q = 0; q < p->n; q++) {
        m.lay[q] = (uint8_t)p->lay_final[q];
        if (q >= m.b) m.cmask |= 1u << p->lay_final[q];
        else m.smask |= 1u << p->lay_final[q];
    }
    m.kc = (uint32_t)__builtin_popcount(m.cmask & ((1u << m.c) - 1u));
    m.part_log = p->part_log;
    m.tiled = p->samp_tiled;
    m.kv = p->samp_kv;
    m.nfree = p->samp_nfree;
    m.tfree = p->samp_tfree;
    std::memcpy(m.bsrc, p->samp_bsrc, sizeof m.bsrc);
    return m;
}

// logical-order bits of a physical mask
static uint32_t to_logical(const tqs_plan *p, uint32_t x) {
    uint32_t r = 0;
    for (uint32_t q = 0; q < p->n; q++) r |= ((x >> p->lay_final[q]) & 1u) << q;
    return r;
}

template <typename R>
static SampleArgs<R> sample_args(const tqs_plan *p, const Layout &Ly, unsigned char *ws, const Task &t,
                                 uint64_t leaf_first) {
    SampleArgs<R> a;
    std::memset(&a, 0, sizeof a);
    const uint32_t *sched = reinterpret_cast<const uint32_t *>(ws + Ly.off_sched);
    a.states = reinterpret_cast<const cplx<R> *>(ws + Ly.off_states);
    a.slot_amps = 1ull << p->n;
    a.slots = sched + t.slot_of();
    a.node_ids = sched + t.node_ids();
    a.rep = sched + t.rep_of();
    a.rep_slots = sched + t.cdst();
    a.reps = t.ccount;
    a.part = reinterpret_cast<double *>(ws + Ly.off_part);
    a.sums = reinterpret_cast<double *>(ws + Ly.off_sums);
    a.leaf_u = reinterpret_cast<const double *>(ws + Ly.off_leafu);
    a.leaf_fx = reinterpret_cast<const uint32_t *>(ws + Ly.off_leaffx);
    a.leaf_flip = reinterpret_cast<const uint32_t *>(ws + Ly.off_flip);
    a.outcomes = reinterpret_cast<uint64_t *>(ws + Ly.off_out);
    a.leaf_first = leaf_first;
    a.leaf_off = (uint32_t)p->level_offset.back();
    a.count = t.count;
    a.m = sample_map(p);
    return a;
}

// Workgroups of the partials / gather / sample launches for one segment.
template <typename R>
static void sample_grid(const SampleArgs<R> &a, uint32_t g[3]) {
    g[0] = a.m.tiled ? 0u : a.reps << (a.m.n - a.m.c);
    {
        // tiled partials: each workgroup takes kThreads >> ls items (ls =
        // log2 of the shares per item), else one item per thread
        const uint32_t nb = (uint32_t)__builtin_popcount(a.m.tfree);
        const uint32_t per = a.m.tiled ? (kThreads >> (nb < 3u ? nb : 3u)) : kThreads;
        g[1] = (uint32_t)((((uint64_t)a.reps << (a.m.n - a.m.b)) + per - 1) / per);
    }
    g[2] = a.count;
}

template <typename R>
static void launch_sample_kernels(const SampleLaunch<R> &sl, const uint32_t grid[3], hipStream_t s) {
    if (grid[0]) hipLaunchKernelGGL(block_partials_kernel<R>, dim3(grid[0]), dim3(kThreads), 0, s, sl);
    hipLaunchKernelGGL(block_gather_kernel<R>, dim3(grid[1]), dim3(kThreads), 0, s, sl);
    hipLaunchKernelGGL(sample_kernel<R>, dim3(grid[2]), dim3(kThreads), 0, s, sl);
}

template <typename R>
static void launch_sample(const tqs_plan *p, const Layout &Ly, unsigned char *ws, hipStream_t s,
                          const Task &t, uint64_t leaf_first) {
    SampleLaunch<R> sl;
    std::memset(&sl, 0, sizeof sl);
    sl.one = sample_args<R>(p, Ly, ws, t, leaf_first);
    uint32_t g[3];
    sample_grid(sl.one, g);
    launch_sample_kernels(sl, g, s);
}

static tqs_status check_noise(const tqs_plan *p, const tqs_noise *nz) {
    if (!nz) return fail(TQS_E_ARG, "noise is NULL");
    if (nz->n_gates != p->n_gates || nz->arity != p->arity || nz->cut != p->cut)
        return fail(TQS_E_ARG, "noise list was sampled for another circuit or tree");
    if (!nz->leaf_flip.empty()) {
        if (nz->leaf_flip.size() != p->n_leaves) return fail(TQS_E_ARG, "read-out flips: one mask per leaf");
        const uint64_t lim = 1ull << p->n;
        for (uint64_t i = 0; i < nz->leaf_flip.size(); i++)
            if (nz->leaf_flip[i] >= lim)
                return fail(TQS_E_ARG, "read-out flip mask of leaf %llu has bits beyond qubit %u",
                            (unsigned long long)i, p->n - 1);
    }
    return TQS_OK;
}

static hipEvent_t pool_event(std::vector<void *> &pool, size_t i) {
    while (pool.size() <= i) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        pool.push_back((void *)e);
    }
    return (hipEvent_t)pool[i];
}

struct Capture {
    const uint64_t *leaves = nullptr;
    uint64_t n = 0;
    double *amps = nullptr;
};

// The plan data, noise metadata and schedule of one run, written into a
// host image of the workspace whose first byte is workspace offset `base`.
template <typename R>
static void pack_meta(const tqs_plan *p, const tqs_noise *nz, const HostMeta &hm,
                      const std::vector<uint32_t> &sched, const Layout &Ly, unsigned char *hb, uint64_t base,
                      const FrameTables *ftab = nullptr) {
    auto put = [&](uint64_t off, const void *src, size_t bytes) {
        if (bytes) std::memcpy(hb + (off - base), src, bytes);
    };
    {
        std::vector<cplx<R>> mats(p->mats.size());
        for (size_t i = 0; i < mats.size(); i++) mats[i] = {(R)p->mats[i].real(), (R)p->mats[i].imag()};
        put(Ly.off_mats, mats.data(), mats.size() * sizeof(cplx<R>));
    }
    put(Ly.off_ops, p->ops.data(), p->ops.size() * sizeof(OpDesc));
    put(Ly.off_passes, p->passes.data(), p->passes.size() * sizeof(PassDesc));
    put(Ly.off_terms, p->terms.data(), p->terms.size() * sizeof(DiagTerm));
    put(Ly.off_dgates, p->dgates.data(), p->dgates.size() * sizeof(DiagGate));
    put(Ly.off_frame0, hm.frame0.data(), hm.frame0.size() * 4);
    put(Ly.off_evoff, hm.ev_off.data(), hm.ev_off.size() * 4);
    put(Ly.off_evpos, hm.ev_pos.data(), hm.ev_pos.size() * 4);
    put(Ly.off_evdx, hm.ev_dx.data(), hm.ev_dx.size() * 4);
    put(Ly.off_evdz, hm.ev_dz.data(), hm.ev_dz.size() * 4);
    put(Ly.off_leafu, nz->leaf_u.data(), nz->leaf_u.size() * 8);
    put(Ly.off_leaffx, hm.leaf_fx.data(), hm.leaf_fx.size() * 4);
    put(Ly.off_flip, nz->leaf_flip.data(), nz->leaf_flip.size() * 4);  // zeros when absent
    put(Ly.off_sched, sched.data(), sched.size() * 4);
    if (ftab) {
        put(Ly.off_ctoff, ftab->ct_off.data(), ftab->ct_off.size() * 4);
        std::vector<cplx<R>> t(ftab->tab.size());
        for (size_t i = 0; i < t.size(); i++) t[i] = {(R)ftab->tab[i].real(), (R)ftab->tab[i].imag()};
        put(Ly.off_ctab, t.data(), t.size() * sizeof(cplx<R>));
    } else {
        std::vector<uint32_t> none(p->n_nodes, 0xFFFFFFFFu);
        put(Ly.off_ctoff, none.data(), none.size() * 4);
    }
}

// A roctx range open for the lifetime of the object (every return path).
struct MarkerRange {
    explicit MarkerRange(const char *name) { roctxRangePush(name); }
    ~MarkerRange() { roctxRangePop(); }
    MarkerRange(const MarkerRange &) = delete;
    MarkerRange &operator=(const MarkerRange &) = delete;
};

// Failure injection for tests of the error paths, set from the environment
// and read on each run; host side only, no kernel is altered.
//   TQS_FAULT=alloc     the host allocation of the run's metadata fails
//                       (TQS_E_OOM) before any device call;
//   TQS_FAULT=launch:K  the run's K-th pass (from 0) reports a launch
//                       failure (TQS_E_HIP) after the passes before it
//                       were enqueued ("launch" alone: K = 0).
struct FaultSpec {
    enum Kind { NONE, ALLOC, LAUNCH } kind = NONE;
    uint64_t at = 0;
};

static FaultSpec fault_spec() {
    FaultSpec f;
    const char *e = std::getenv("TQS_FAULT");
    if (!e || !*e) return f;
    if (!std::strcmp(e, "alloc")) {
        f.kind = FaultSpec::ALLOC;
    } else if (!std::strncmp(e, "launch", 6) && (e[6] == 0 || e[6] == ':')) {
        f.kind = FaultSpec::LAUNCH;
        if (e[6] == ':') f.at = std::strtoull(e + 7, nullptr, 10);
    }
    return f;
}

// A run that fails after it enqueued device work waits for that work before
// returning, so the caller may free or reuse the workspace at once.
struct DrainOnError {
    hipStream_t s;
    bool armed = false;
    explicit DrainOnError(hipStream_t st) : s(st) {}
    ~DrainOnError() {
        if (armed) (void)hipStreamSynchronize(s);
    }
    DrainOnError(const DrainOnError &) = delete;
    DrainOnError &operator=(const DrainOnError &) = delete;
};

}  // namespace tqs

// A run between tqs_run_start and tqs_run_finish: its staging slot, the
// launch counts and the events its statistics are read from.
struct tqs_pending {
    tqs_plan *p = nullptr;
    int slot = -1;
    hipStream_t s = nullptr;
    uint64_t *outcomes = nullptr;
    uint64_t n_out = 0;
    bool stats = false;
    std::chrono::steady_clock::time_point t0;
    uint64_t launches = 0, pass_launches = 0, pass_states = 0, bytes_passes = 0, bytes_sample = 0, merged = 0;
    uint64_t jit_launches = 0, jit_states = 0, bytes_jit = 0, events = 0;
    hipEvent_t e_begin = nullptr, e_end = nullptr;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> jit_ev, pass_ev, samp_ev;
    std::vector<unsigned char> meta;  // the uploaded metadata of a run without a staging slot
};

namespace tqs {

// A free staging slot of the plan (*k) with pinned buffers of at least the
// given sizes, marked busy; TQS_E_ARG when both are in use.
static tqs_status acquire_slot(tqs_plan *p, uint64_t meta_bytes, uint64_t out_bytes, int *k) {
    *k = -1;
    {
        std::lock_guard<std::mutex> lock(p->slot_mu);
        for (int i = 0; i < 2 && *k < 0; i++)
            if (!p->slots[i].busy) {
                p->slots[i].busy = true;
                *k = i;
            }
    }
    if (*k < 0) return fail(TQS_E_ARG, "two runs of this plan are already in flight (finish one first)");
    tqs_plan::RunSlot &sl = p->slots[*k];
    auto grow = [](void **buf, uint64_t *cap, uint64_t need) {
        if (*cap >= need) return true;
        if (*buf) (void)hipHostFree(*buf);
        *buf = nullptr;
        *cap = 0;
        const uint64_t want = std::max<uint64_t>(need, 1ull << 16);
        if (hipHostMalloc(buf, want, hipHostMallocDefault) != hipSuccess) {
            *buf = nullptr;
            return false;
        }
        *cap = want;
        return true;
    };
    if (!grow(&sl.meta, &sl.meta_cap, meta_bytes) || !grow(&sl.out, &sl.out_cap, out_bytes)) {
        std::lock_guard<std::mutex> lock(p->slot_mu);
        sl.busy = false;
        *k = -1;
        return fail(TQS_E_OOM, "pinned host staging allocation failed");
    }
    return TQS_OK;
}

static void release_slot(tqs_plan *p, int k) {
    if (k < 0) return;
    std::lock_guard<std::mutex> lock(p->slot_mu);
    p->slots[k].busy = false;
}

// Frees a started run's slot unless the run was handed over (done).
struct SlotGuard {
    tqs_plan *p;
    int k = -1;
    bool done = false;
    ~SlotGuard() {
        if (!done) release_slot(p, k);
    }
};

// Everything of a run up to its outcome download, enqueued on the stream:
// the host prologue (noise metadata, schedule, routing, packing into the
// slot's pinned buffer), the upload, every pass and sampling launch, and
// the download into the slot's pinned buffer.  Returns without waiting
// (capture requests aside, which copy leaf states out as they come).
// noalloc: no host or device allocation through HIP (tqs_run_noalloc): the
// metadata goes up from pageable memory and the outcomes come straight down
// (both copies then wait for the stream), no staging slot, and the plan's
// specialised kernels only if they are already loaded on this device (else
// the generic kernels take every state).
template <typename R>
static tqs_status run_start_t(tqs_plan *p, const tqs_noise *nz, unsigned char *ws, uint64_t ws_bytes,
                              hipStream_t s, uint64_t first, uint64_t last, uint64_t *outcomes,
                              bool stats, const Capture &cap, tqs_pending *pd, bool noalloc) {
    const auto t0 = std::chrono::steady_clock::now();
    tqs_status st = check_noise(p, nz);
    if (st) return st;
    if (first >= last || last > p->arity[0])
        return fail(TQS_E_ARG, "subtree range [%llu, %llu) outside [0, %llu)", (unsigned long long)first,
                    (unsigned long long)last, (unsigned long long)p->arity[0]);
    if (!outcomes) return fail(TQS_E_ARG, "outcomes is NULL");
    if (!ws) return fail(TQS_E_WORKSPACE, "workspace is NULL");
    if (((uintptr_t)ws) & 255) return fail(TQS_E_WORKSPACE, "workspace must be 256-byte aligned");
    const uint32_t L = (uint32_t)p->arity.size();
    uint64_t per_subtree = 1;
    for (uint32_t l = 1; l < L; l++) per_subtree *= p->arity[l];
    const uint64_t leaf_first = first * per_subtree;
    const uint64_t n_out = (last - first) * per_subtree;

    const FaultSpec fault = fault_spec();
    if (fault.kind == FaultSpec::ALLOC) throw std::bad_alloc();
    HostMeta hm;
    build_meta(p, nz, &hm);
    std::vector<Task> tasks;
    std::vector<uint32_t> sched;
    Layout Ly0 = make_layout(p, nz->ev_gate.size(), n_out, 0);
    build_schedule(p, first, last, &tasks, &sched, Ly0.slot_base, p->tune.no_merge ? nullptr : &hm);
    bool use_jit = p->tune.jit == 1;
    if (use_jit && noalloc) {
        int dev = -1;
        use_jit = hipGetDevice(&dev) == hipSuccess && p->jit_module && p->jit_device == dev;
    }
    if (use_jit) {
        // the plan's specialised kernels, compiled on its first run
        const tqs_status js = jit_prepare(p);
        if (js) return js;
    }
    std::vector<std::vector<Route>> routes;
    FrameTables ftab;
    route_passes(p, hm, tasks, &sched, &routes, &ftab, use_jit);
    Layout Ly = make_layout(p, nz->ev_gate.size(), n_out, sched.size(), 0, ~0ull, ftab.tab.size());
    if (ws_bytes < Ly.total)
        return fail(TQS_E_WORKSPACE, "workspace has %llu bytes, the run needs %llu",
                    (unsigned long long)ws_bytes, (unsigned long long)Ly.total);

    // pack the metadata exactly as laid out in the workspace, into the
    // slot's pinned buffer
    const uint64_t meta_bytes = Ly.off_sums - Ly.off_meta;
    SlotGuard sg{p};
    std::vector<void *> direct_events;  // (event pool of a run without a slot)
    unsigned char *hb = nullptr;
    if (noalloc) {
        pd->meta.assign(meta_bytes, 0);
        hb = pd->meta.data();
    } else {
        st = acquire_slot(p, meta_bytes, n_out * 8, &sg.k);
        if (st) return st;
        hb = static_cast<unsigned char *>(p->slots[sg.k].meta);
        std::memset(hb, 0, meta_bytes);
    }
    std::vector<void *> &ev_pool = noalloc ? direct_events : p->slots[sg.k].events;
    pack_meta<R>(p, nz, hm, sched, Ly, hb, Ly.off_meta, &ftab);

    DrainOnError drain(s);
    drain.armed = true;
    size_t ev_i = 0;
    hipEvent_t e_begin = nullptr, e_end = nullptr;
    if (stats) {
        e_begin = pool_event(ev_pool, ev_i++);
        if (!e_begin) return fail(TQS_E_HIP, "hipEventCreate failed");
        HIP_TRY(hipEventRecord(e_begin, s), "hipEventRecord");
    }
    HIP_TRY(hipMemcpyAsync(ws + Ly.off_meta, hb, meta_bytes, hipMemcpyHostToDevice, s), "metadata upload");

    // capture requests: leaf -> capture indices
    std::vector<std::vector<uint64_t>> cap_of;
    std::vector<unsigned char> cap_host;
    if (cap.n) {
        cap_host.resize(Ly.state_bytes);
    }

    uint64_t launches = 0, pass_launches = 0, pass_states = 0, bytes_passes = 0, bytes_sample = 0, merged = 0;
    uint64_t jit_launches = 0, jit_states = 0, bytes_jit = 0, pass_iter = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> jit_ev;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pass_ev, samp_ev;
    const uint64_t state_bytes = Ly.state_bytes;
    const uint32_t b = p->sample_b;
    for (const Task &t : tasks) {
        const tqs::Level &lv = p->levels[t.level];
        merged += t.count - t.ccount;
        // a marker range per chunk task, for timelines (no cost without a tool)
        char mark[64];
        std::snprintf(mark, sizeof mark, "tqs level %u: %u nodes, %u computed", t.level, t.count, t.ccount);
        const MarkerRange range(mark);
        hipEvent_t ea = nullptr, eb = nullptr, ec = nullptr;
        if (stats) {
            ea = pool_event(ev_pool, ev_i++);
            eb = pool_event(ev_pool, ev_i++);
            if (!ea || !eb) return fail(TQS_E_HIP, "hipEventCreate failed");
            HIP_TRY(hipEventRecord(ea, s), "hipEventRecord");
        }
        const LevelShape lsh = level_shape(p, t.level);
        if constexpr (sizeof(R) == 4) if (lsh.waves && t.ccount) {
            // the whole level in one launch, the states in LDS between passes
            if (fault.kind == FaultSpec::LAUNCH && pass_iter <= fault.at && fault.at < pass_iter + lv.pass_count)
                HIP_TRY(hipErrorLaunchFailure, "pass launch (TQS_FAULT)");
            pass_iter += lv.pass_count;
            LevelLaunch<float> ll;
            std::memset(&ll, 0, sizeof ll);
            ll.a = pass_args<float>(p, Ly, ws, t, lv.pass_begin, true);
            ll.npass = lv.pass_count;
            const PassArgs<float> al = pass_args<float>(p, Ly, ws, t, lv.pass_begin + lv.pass_count - 1, false);
            ll.part = al.part;
            ll.psum = al.psum;
            bool d2 = false;
            for (uint32_t k = 0; k < lv.pass_count; k++) d2 = d2 || p->passes[lv.pass_begin + k].has_d2;
            launch_level_kernel(p->reg_bits, d2, ll, lsh.waves, lsh.lds, s);
            HIP_TRY(hipGetLastError(), "level kernel launch");
            launches++;
            pass_launches++;
            pass_states += t.ccount;
            const bool init = t.level == 0;
            const bool parts = p->samp_tiled && t.level == L - 1;
            bytes_passes += (uint64_t)t.ccount * (state_bytes * (init ? 1 : 2) +
                                                  (parts ? (8ull << (p->samp_nfree + p->samp_kv)) : 0ull));
        }
        for (uint32_t k = 0; k < (lsh.waves ? 0u : lv.pass_count); k++) {
            uint32_t nl = 0;
            hipError_t le = hipSuccess;
            hipEvent_t ej0 = nullptr, ej1 = nullptr;
            if (stats) {
                // the specialised launch of this pass, timed on its own
                ej0 = pool_event(ev_pool, ev_i++);
                ej1 = pool_event(ev_pool, ev_i++);
                if (!ej0 || !ej1) return fail(TQS_E_HIP, "hipEventCreate failed");
            }
            if (fault.kind == FaultSpec::LAUNCH && pass_iter == fault.at)
                HIP_TRY(hipErrorLaunchFailure, "pass launch (TQS_FAULT)");
            pass_iter++;
            const uint32_t nj = launch_routed<R>(p, Ly, ws, s, t, lv.pass_begin + k, k == 0,
                                                 routes[&t - tasks.data()][k], &nl, &le, ej0, ej1);
            HIP_TRY(le, "specialised pass kernel launch");
            launches += nl;
            pass_launches += nl;
            pass_states += t.ccount;
            const bool init = (k == 0 && t.level == 0);
            const bool parts = p->samp_tiled && t.level == L - 1 && k + 1 == lv.pass_count;
            // algorithmic bytes per computed state: one read and one write
            // (write only for the generated |0..0>), plus its sampling partials
            const uint64_t per_state =
                state_bytes * (init ? 1 : 2) + (parts ? (8ull << (p->samp_nfree + p->samp_kv)) : 0ull);
            bytes_passes += (uint64_t)t.ccount * per_state;
            if (nj) {
                jit_launches++;
                jit_states += nj;
                bytes_jit += (uint64_t)nj * per_state;
                if (stats) jit_ev.push_back({ej0, ej1});
            }
        }
        if (stats) {
            HIP_TRY(hipEventRecord(eb, s), "hipEventRecord");
            pass_ev.push_back({ea, eb});
        }
        if (t.level == L - 1) {
            launch_sample<R>(p, Ly, ws, s, t, leaf_first);
            launches += 3;
            // partial masses (the states themselves when the pass wrote none),
            // then one block of each leaf
            bytes_sample += (uint64_t)t.ccount * (p->samp_tiled ? (8ull << (p->samp_nfree + p->samp_kv)) : state_bytes) +
                            (uint64_t)t.count * (Ly.amp_bytes << b);
            if (stats) {
                ec = pool_event(ev_pool, ev_i++);
                if (!ec) return fail(TQS_E_HIP, "hipEventCreate failed");
                HIP_TRY(hipEventRecord(ec, s), "hipEventRecord");
                samp_ev.push_back({eb, ec});
            }
            if (cap.n) {
                // materialise the frame of requested leaves (standalone Pauli
                // application into the scratch slot) and copy them out
                for (uint32_t i = 0; i < t.count; i++) {
                    const uint64_t lam = t.first + i;
                    for (uint64_t ci = 0; ci < cap.n; ci++) {
                        if (cap.leaves[ci] != lam) continue;
                        const Frame &f = hm.leaf_frame[lam];
                        const uint32_t slot = sched[t.slot_of() + i];
                        const uint64_t amps = 1ull << p->n;
                        const cplx<R> *in = reinterpret_cast<const cplx<R> *>(ws + Ly.off_states) + (uint64_t)slot * amps;
                        cplx<R> *out = reinterpret_cast<cplx<R> *>(ws + Ly.off_states) + (uint64_t)Ly.scratch_slot * amps;
                        hipLaunchKernelGGL(frame_apply_kernel<R>, dim3((uint32_t)((amps + kThreads - 1) / kThreads)),
                                           dim3(kThreads), 0, s, in, out, amps, f.x, f.z, f.k, sample_map(p));
                        HIP_TRY(hipGetLastError(), "frame_apply launch");
                        HIP_TRY(hipMemcpyAsync(cap_host.data(), out, state_bytes, hipMemcpyDeviceToHost, s),
                                "capture copy");
                        HIP_TRY(hipStreamSynchronize(s), "capture sync");
                        const cplx<R> *h = reinterpret_cast<const cplx<R> *>(cap_host.data());
                        double *dstp = cap.amps + ci * 2 * amps;
                        for (uint64_t y = 0; y < amps; y++) {
                            dstp[2 * y] = (double)h[y].re;
                            dstp[2 * y + 1] = (double)h[y].im;
                        }
                    }
                }
            }
        }
        HIP_TRY(hipGetLastError(), "kernel launch");
    }
    HIP_TRY(hipMemcpyAsync(noalloc ? (void *)outcomes : p->slots[sg.k].out, ws + Ly.off_out, n_out * 8,
                           hipMemcpyDeviceToHost, s),
            "outcome download");
    if (stats) {
        e_end = pool_event(ev_pool, ev_i++);
        if (!e_end) return fail(TQS_E_HIP, "hipEventCreate failed");
        HIP_TRY(hipEventRecord(e_end, s), "hipEventRecord");
    }
    // the run is enqueued: the pending record owns its slot from here
    pd->p = p;
    pd->slot = sg.k;
    pd->s = s;
    pd->outcomes = outcomes;
    pd->n_out = n_out;
    pd->stats = stats;
    pd->t0 = t0;
    pd->launches = launches;
    pd->pass_launches = pass_launches;
    pd->pass_states = pass_states;
    pd->bytes_passes = bytes_passes;
    pd->bytes_sample = bytes_sample;
    pd->merged = merged;
    pd->jit_launches = jit_launches;
    pd->jit_states = jit_states;
    pd->bytes_jit = bytes_jit;
    pd->events = nz->ev_gate.size();
    pd->e_begin = e_begin;
    pd->e_end = e_end;
    pd->jit_ev = std::move(jit_ev);
    pd->pass_ev = std::move(pass_ev);
    pd->samp_ev = std::move(samp_ev);
    sg.done = true;
    drain.armed = false;
    return TQS_OK;
}

// Wait for a started run, copy its outcomes out and read its statistics;
// the slot is free again whatever happens.
static tqs_status run_finish(tqs_pending *pd, tqs_run_stats *stats) {
    SlotGuard sg{pd->p};
    sg.k = pd->slot;
    HIP_TRY(hipStreamSynchronize(pd->s), "stream synchronize");
    if (pd->slot >= 0) std::memcpy(pd->outcomes, pd->p->slots[pd->slot].out, pd->n_out * 8);
    if (stats) {
        std::memset(stats, 0, sizeof *stats);
        if (pd->stats) {
            float ms = 0;
            HIP_TRY(hipEventElapsedTime(&ms, pd->e_begin, pd->e_end), "hipEventElapsedTime");
            stats->ms_device = ms;
            for (auto &pr : pd->pass_ev) {
                HIP_TRY(hipEventElapsedTime(&ms, pr.first, pr.second), "hipEventElapsedTime");
                stats->ms_passes += ms;
            }
            for (auto &pr : pd->samp_ev) {
                HIP_TRY(hipEventElapsedTime(&ms, pr.first, pr.second), "hipEventElapsedTime");
                stats->ms_sample += ms;
            }
            for (auto &pr : pd->jit_ev) {
                HIP_TRY(hipEventElapsedTime(&ms, pr.first, pr.second), "hipEventElapsedTime");
                stats->ms_jit += ms;
            }
        }
        stats->launches = pd->launches;
        stats->pass_launches = pd->pass_launches;
        stats->pass_states = pd->pass_states;
        stats->bytes_passes = pd->bytes_passes;
        stats->bytes_sample = pd->bytes_sample;
        stats->events = pd->events;
        stats->nodes_merged = pd->merged;
        stats->jit_launches = pd->jit_launches;
        stats->jit_states = pd->jit_states;
        stats->bytes_jit = pd->bytes_jit;
        stats->ms_wall = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - pd->t0).count();
    }
    return TQS_OK;
}

static tqs_status run_start_any(tqs_plan *p, const tqs_noise *nz, void *ws, uint64_t ws_bytes, void *stream,
                                uint64_t first, uint64_t last, uint64_t *outcomes, bool stats, const Capture &cap,
                                tqs_pending *pd, bool noalloc = false) {
    if (!p) return fail(TQS_E_ARG, "plan is NULL");
    hipStream_t s = (hipStream_t)stream;
    if (p->prec == TQS_C64)
        return run_start_t<float>(p, nz, (unsigned char *)ws, ws_bytes, s, first, last, outcomes, stats, cap, pd,
                                  noalloc);
    return run_start_t<double>(p, nz, (unsigned char *)ws, ws_bytes, s, first, last, outcomes, stats, cap, pd,
                               noalloc);
}

// A whole run: started, then finished at once.
static tqs_status run_any(tqs_plan *p, const tqs_noise *nz, void *ws, uint64_t ws_bytes, void *stream,
                          uint64_t first, uint64_t last, uint64_t *outcomes, tqs_run_stats *stats,
                          const Capture &cap, bool noalloc = false) {
    tqs_pending pd;
    const tqs_status st =
        run_start_any(p, nz, ws, ws_bytes, stream, first, last, outcomes, stats != nullptr, cap, &pd, noalloc);
    if (st) return st;
    return run_finish(&pd, stats);
}

// ------------------------------------------------------------- batches --
// Several independent runs (different circuits, trees, noise) advanced
// together: run i's k-th launch (a pass over a chunk of states, or the
// sampling of a leaf chunk) goes into step k, and each step is one pass
// launch and one sampling launch whose segments are the runs' launches, so
// small circuits share the device instead of queueing one small grid after
// another.  Within a run the launches keep their order; runs never share
// state slots.
struct BatchOp {
    uint32_t kind;  // 0 pass, 1 sampling
    uint32_t task, pass, first;
};

struct BatchItem {
    tqs_plan *p = nullptr;
    const tqs_noise *nz = nullptr;
    Layout Ly;
    HostMeta hm;
    std::vector<Task> tasks;
    std::vector<uint32_t> sched;
    std::vector<BatchOp> ops;
    uint64_t leaf_base = 0;
};

}  // namespace tqs

struct tqs_batch {
    tqs_precision prec = TQS_C64;
    uint32_t reg_bits = 0;
    std::vector<tqs::BatchItem> items;
    uint32_t steps = 0;
    std::vector<uint32_t> npass, nsamp;  // segments per step
    uint64_t table_at = 0, table_bytes = 0, total = 0, leaves = 0;
    std::vector<void *> events;
    // launch replay: the steps' kernels recorded once into a HIP graph on a
    // private stream, for the workspace they were recorded with
    bool use_graph = false;
    void *graph_exec = nullptr;    // hipGraphExec_t
    void *capture_stream = nullptr;  // hipStream_t
    const unsigned char *graph_ws = nullptr;
};

namespace tqs {

template <typename R>
static tqs_status batch_run_t(tqs_batch *B, unsigned char *ws, uint64_t ws_bytes, hipStream_t s,
                              uint64_t *outcomes, tqs_run_stats *stats) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!ws) return fail(TQS_E_WORKSPACE, "workspace is NULL");
    if (((uintptr_t)ws) & 255) return fail(TQS_E_WORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < B->total)
        return fail(TQS_E_WORKSPACE, "workspace has %llu bytes, the batch needs %llu",
                    (unsigned long long)ws_bytes, (unsigned long long)B->total);
    if (!outcomes) return fail(TQS_E_ARG, "outcomes is NULL");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (stats) {
        while (B->events.size() < 2) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) return fail(TQS_E_HIP, "hipEventCreate failed");
            B->events.push_back((void *)e);
        }
        e0 = (hipEvent_t)B->events[0];
        e1 = (hipEvent_t)B->events[1];
        HIP_TRY(hipEventRecord(e0, s), "hipEventRecord");
    }
    // per-run metadata
    std::vector<std::vector<unsigned char>> hbs(B->items.size());
    for (size_t i = 0; i < B->items.size(); i++) {
        BatchItem &it = B->items[i];
        hbs[i].assign(it.Ly.off_sums - it.Ly.off_meta, 0);
        pack_meta<R>(it.p, it.nz, it.hm, it.sched, it.Ly, hbs[i].data(), it.Ly.off_meta);
        HIP_TRY(hipMemcpyAsync(ws + it.Ly.off_meta, hbs[i].data(), hbs[i].size(), hipMemcpyHostToDevice, s),
                "metadata upload");
    }
    // segment tables of every step
    std::vector<unsigned char> tb(B->table_bytes, 0);
    std::vector<uint64_t> pass_at(B->steps), samp_at(B->steps);
    std::vector<uint32_t> pass_total(B->steps, 0), pass_d2(B->steps, 0);
    std::vector<std::array<uint32_t, 3>> samp_total(B->steps, {0, 0, 0});
    {
        uint64_t o = 0;
        for (uint32_t k = 0; k < B->steps; k++) {
            pass_at[k] = o;
            PassArgs<R> *pa = reinterpret_cast<PassArgs<R> *>(tb.data() + o);
            o += align256((uint64_t)B->npass[k] * sizeof(PassArgs<R>));
            samp_at[k] = o;
            SampleArgs<R> *sa = reinterpret_cast<SampleArgs<R> *>(tb.data() + o);
            o += align256((uint64_t)B->nsamp[k] * sizeof(SampleArgs<R>));
            uint32_t np = 0, ns = 0;
            for (BatchItem &it : B->items) {
                if (k >= it.ops.size()) continue;
                const BatchOp &op = it.ops[k];
                const Task &t = it.tasks[op.task];
                if (op.kind == 0) {
                    PassArgs<R> a = pass_args<R>(it.p, it.Ly, ws, t, op.pass, op.first != 0);
                    a.wg_begin = pass_total[k];
                    pass_total[k] += a.work;
                    if (it.p->passes[op.pass].has_d2) pass_d2[k] = 1;
                    pa[np++] = a;
                } else {
                    SampleArgs<R> a = sample_args<R>(it.p, it.Ly, ws, t, 0);
                    uint32_t g[3];
                    sample_grid(a, g);
                    for (int q = 0; q < 3; q++) {
                        a.wg_begin[q] = samp_total[k][q];
                        samp_total[k][q] += g[q];
                    }
                    sa[ns++] = a;
                }
            }
        }
    }
    DrainOnError drain(s);
    drain.armed = true;
    HIP_TRY(hipMemcpyAsync(ws + B->table_at, tb.data(), tb.size(), hipMemcpyHostToDevice, s), "table upload");
    // the kernel arguments depend only on the batch and the workspace
    // address, so one recording serves every later run with that workspace
    auto launch_steps = [&](hipStream_t ls) -> tqs_status {
        for (uint32_t k = 0; k < B->steps; k++) {
            if (B->npass[k]) {
                PassLaunch<R> pl;
                std::memset(&pl, 0, sizeof pl);
                pl.segs = reinterpret_cast<const PassArgs<R> *>(ws + B->table_at + pass_at[k]);
                pl.nseg = B->npass[k];
                pl.total = pass_total[k];
                launch_pass_kernel<R>(B->reg_bits, pass_d2[k] != 0, pl, ls);
            }
            if (B->nsamp[k]) {
                SampleLaunch<R> sl;
                std::memset(&sl, 0, sizeof sl);
                sl.segs = reinterpret_cast<const SampleArgs<R> *>(ws + B->table_at + samp_at[k]);
                sl.nseg = B->nsamp[k];
                const uint32_t g[3] = {samp_total[k][0], samp_total[k][1], samp_total[k][2]};
                launch_sample_kernels(sl, g, ls);
            }
            HIP_TRY(hipGetLastError(), "kernel launch");
        }
        return TQS_OK;
    };
    if (B->use_graph) {
        if (!B->graph_exec || B->graph_ws != ws) {
            if (B->graph_exec) {
                (void)hipGraphExecDestroy((hipGraphExec_t)B->graph_exec);
                B->graph_exec = nullptr;
            }
            if (!B->capture_stream) {
                hipStream_t cs = nullptr;
                HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreate");
                B->capture_stream = (void *)cs;
            }
            hipStream_t cs = (hipStream_t)B->capture_stream;
            HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed), "hipStreamBeginCapture");
            tqs_status st = launch_steps(cs);
            hipGraph_t g = nullptr;
            const hipError_t ec = hipStreamEndCapture(cs, &g);
            if (st) {
                if (g) (void)hipGraphDestroy(g);
                return st;
            }
            HIP_TRY(ec, "hipStreamEndCapture");
            hipGraphExec_t ex = nullptr;
            const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            HIP_TRY(ei, "hipGraphInstantiate");
            B->graph_exec = (void *)ex;
            B->graph_ws = ws;
        }
        HIP_TRY(hipGraphLaunch((hipGraphExec_t)B->graph_exec, s), "hipGraphLaunch");
    } else {
        tqs_status st = launch_steps(s);
        if (st) return st;
    }
    for (BatchItem &it : B->items)
        HIP_TRY(hipMemcpyAsync(outcomes + it.leaf_base, ws + it.Ly.off_out, it.p->n_leaves * 8,
                               hipMemcpyDeviceToHost, s),
                "outcome download");
    if (stats) HIP_TRY(hipEventRecord(e1, s), "hipEventRecord");
    HIP_TRY(hipStreamSynchronize(s), "stream synchronize");
    drain.armed = false;
    if (stats) {
        std::memset(stats, 0, sizeof *stats);
        float ms = 0;
        HIP_TRY(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
        stats->ms_device = ms;
        uint64_t launches = 0;
        for (uint32_t k = 0; k < B->steps; k++) launches += (B->npass[k] ? 1 : 0) + (B->nsamp[k] ? 3 : 0);
        stats->launches = launches;
        stats->ms_wall =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return TQS_OK;
}

}  // namespace tqs

using namespace tqs;

tqs_plan::~tqs_plan() {
    for (RunSlot &sl : slots) {
        for (void *e : sl.events) (void)hipEventDestroy((hipEvent_t)e);
        if (sl.meta) (void)hipHostFree(sl.meta);
        if (sl.out) (void)hipHostFree(sl.out);
    }
    jit_release(this);
}

// ----------------------------------------------- run without allocation --
// For callers that cannot allocate device memory: the run's workspace is a
// file-scope device array of kStaticScratchBytes, one copy per GPU, held
// until the process ends.  Host code never passes the array's name to a
// kernel or a copy (on the host it is not a device address): each device's
// address comes from hipGetSymbolAddress, taken once per device on its
// first call with that device current.
constexpr uint64_t kStaticScratchBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace tqs {
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {nullptr};

// The address of this device's scratch array (set up on first use).
static tqs_status scratch_address(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(TQS_E_ARG, "device %d outside 0..%d", dev, kMaxDevices - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!ptr || (((uintptr_t)ptr) & 255)) return fail(TQS_E_HIP, "scratch array address not 256-byte aligned");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return TQS_OK;
}
}  // namespace tqs

#define TQS_GUARD_BEGIN try {
#define TQS_GUARD_END                                         \
    }                                                         \
    catch (const std::bad_alloc &) {                          \
        return fail(TQS_E_OOM, "host allocation failed");     \
    }                                                         \
    catch (...) {                                             \
        return fail(TQS_E_ARG, "unexpected exception");       \
    }

extern "C" {

tqs_status tqs_workspace_bytes(const tqs_plan *p, const tqs_noise *nz, uint64_t *bytes) {
    TQS_GUARD_BEGIN
    if (!p || !bytes) return fail(TQS_E_ARG, "plan or bytes is NULL");
    if (nz) {
        // exact: the schedule of this list (merged states shorten it)
        tqs_status st = check_noise(p, nz);
        if (st) return st;
        HostMeta hm;
        build_meta(p, nz, &hm);
        std::vector<Task> tasks;
        std::vector<uint32_t> sched;
        Layout Ly0 = make_layout(p, nz->ev_gate.size(), p->n_leaves, 0);
        build_schedule(p, 0, p->arity[0], &tasks, &sched, Ly0.slot_base, p->tune.no_merge ? nullptr : &hm);
        std::vector<std::vector<Route>> routes;
        FrameTables ftab;
        route_passes(p, hm, tasks, &sched, &routes, &ftab);
        *bytes = make_layout(p, nz->ev_gate.size(), p->n_leaves, sched.size(), 0, ~0ull, ftab.tab.size()).total;
        return TQS_OK;
    }
    uint64_t ev = 0;
    for (size_t l = 0; l < p->arity.size(); l++) ev += p->level_nodes[l] * (uint64_t)(p->cut[l + 1] - p->cut[l]);
    Layout Ly = make_layout(p, ev, p->n_leaves, 6 * p->n_nodes + route_bound(p), 0, ~0ull, table_bound(p));
    *bytes = Ly.total;
    return TQS_OK;
    TQS_GUARD_END
}

tqs_status tqs_run(tqs_plan *p, const tqs_noise *nz, void *d_workspace, uint64_t ws_bytes, void *stream,
                   uint64_t *outcomes, tqs_run_stats *stats) {
    TQS_GUARD_BEGIN
    if (!p) return fail(TQS_E_ARG, "plan is NULL");
    return run_any(p, nz, d_workspace, ws_bytes, stream, 0, p->arity[0], outcomes, stats, Capture());
    TQS_GUARD_END
}

tqs_status tqs_run_range(tqs_plan *p, const tqs_noise *nz, void *d_workspace, uint64_t ws_bytes,
                         void *stream, uint64_t first, uint64_t last, uint64_t *outcomes,
                         tqs_run_stats *stats) {
    TQS_GUARD_BEGIN
    return run_any(p, nz, d_workspace, ws_bytes, stream, first, last, outcomes, stats, Capture());
    TQS_GUARD_END
}

tqs_status tqs_run_start(tqs_plan *p, const tqs_noise *nz, void *d_workspace, uint64_t ws_bytes, void *stream,
                         uint64_t *outcomes, uint32_t flags, tqs_pending **out) {
    TQS_GUARD_BEGIN
    if (!out) return fail(TQS_E_ARG, "out is NULL");
    *out = nullptr;
    if (!p) return fail(TQS_E_ARG, "plan is NULL");
    if (flags & ~(uint32_t)TQS_RUN_STATS) return fail(TQS_E_ARG, "unknown flags 0x%x", flags);
    std::unique_ptr<tqs_pending> pd(new tqs_pending);
    const tqs_status st = run_start_any(p, nz, d_workspace, ws_bytes, stream, 0, p->arity[0], outcomes,
                                        (flags & TQS_RUN_STATS) != 0, Capture(), pd.get());
    if (st) return st;
    *out = pd.release();
    return TQS_OK;
    TQS_GUARD_END
}

tqs_status tqs_run_finish(tqs_pending *r, tqs_run_stats *stats) {
    TQS_GUARD_BEGIN
    if (!r) return fail(TQS_E_ARG, "run is NULL");
    std::unique_ptr<tqs_pending> pd(r);
    return run_finish(pd.get(), stats);
    TQS_GUARD_END
}

tqs_status tqs_run_capture(tqs_plan *p, const tqs_noise *nz, void *d_workspace, uint64_t ws_bytes,
                           void *stream, uint64_t *outcomes, const uint64_t *leaves, uint64_t n,
                           double *host_amps) {
    TQS_GUARD_BEGIN
    if (!p) return fail(TQS_E_ARG, "plan is NULL");
    if (n && (!leaves || !host_amps)) return fail(TQS_E_ARG, "leaves or host_amps is NULL");
    for (uint64_t i = 0; i < n; i++)
        if (leaves[i] >= p->n_leaves) return fail(TQS_E_ARG, "leaf %llu out of range", (unsigned long long)leaves[i]);
    Capture cap;
    cap.leaves = leaves;
    cap.n = n;
    cap.amps = host_amps;
    return run_any(p, nz, d_workspace, ws_bytes, stream, 0, p->arity[0], outcomes, nullptr, cap);
    TQS_GUARD_END
}

tqs_status tqs_probe_copy(void *d_workspace, uint64_t bytes, uint32_t reps, void *stream, double *gbps) {
    TQS_GUARD_BEGIN
    if (!d_workspace || !gbps || reps < 1 || bytes < 4096 || (bytes & 15))
        return fail(TQS_E_ARG, "bad probe arguments");
    if (((uintptr_t)d_workspace) & 255) return fail(TQS_E_WORKSPACE, "workspace must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    const uint4 *in = (const uint4 *)d_workspace;
    uint4 *out = (uint4 *)((unsigned char *)d_workspace + bytes);
    const uint64_t n16 = bytes / 16;
    const uint32_t grid = (uint32_t)std::min<uint64_t>((n16 + kThreads - 1) / kThreads, 256u * 16u);
    hipEvent_t a, b;
    HIP_TRY(hipEventCreate(&a), "hipEventCreate");
    HIP_TRY(hipEventCreate(&b), "hipEventCreate");
    hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(kThreads), 0, s, in, out, n16);
    HIP_TRY(hipEventRecord(a, s), "hipEventRecord");
    for (uint32_t r = 0; r < reps; r++) hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(kThreads), 0, s, in, out, n16);
    HIP_TRY(hipEventRecord(b, s), "hipEventRecord");
    HIP_TRY(hipEventSynchronize(b), "hipEventSynchronize");
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, a, b), "hipEventElapsedTime");
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *gbps = 2.0 * (double)bytes * reps / (ms * 1e-3) / 1e9;
    return TQS_OK;
    TQS_GUARD_END
}

tqs_status tqs_run_noalloc(tqs_plan *p, const tqs_noise *nz, void *stream, uint64_t *outcomes) {
    TQS_GUARD_BEGIN
    if (!p) return fail(TQS_E_ARG, "plan is NULL");
    hipStream_t s = (hipStream_t)stream;
    int cur = -1;
    HIP_TRY(hipGetDevice(&cur), "hipGetDevice");
    if (s) {
        int sdev = -1;
        HIP_TRY(hipStreamGetDevice(s, &sdev), "hipStreamGetDevice");
        if (sdev != cur) return fail(TQS_E_ARG, "the stream's device %d is not the current device %d", sdev, cur);
    }
    uint64_t need = 0;
    tqs_status st = tqs_workspace_bytes(p, nz, &need);
    if (st) return st;
    if (need > kStaticScratchBytes)
        return fail(TQS_E_WORKSPACE,
                    "the run needs %llu bytes of device memory, more than the library's static scratch "
                    "of %llu bytes (use tqs_run with a workspace)",
                    (unsigned long long)need, (unsigned long long)kStaticScratchBytes);
    void *ws = nullptr;
    st = scratch_address(cur, &ws);
    if (st) return st;
    return run_any(p, nz, ws, kStaticScratchBytes, stream, 0, p->arity[0], outcomes, nullptr, Capture(), true);
    TQS_GUARD_END
}

}  // extern "C"

extern "C" tqs_status tqs_batch_create(tqs_plan *const *plans, const tqs_noise *const *noises, uint32_t count,
                                       tqs_batch **out) {
    TQS_GUARD_BEGIN
    if (!out) return fail(TQS_E_ARG, "out is NULL");
    *out = nullptr;
    if (!plans || !noises || !count) return fail(TQS_E_ARG, "empty batch");
    tqs_batch *B = new tqs_batch;
    B->prec = plans[0] ? plans[0]->prec : TQS_C64;
    B->reg_bits = plans[0] ? plans[0]->reg_bits : 0;
    uint64_t states = 0;
    B->items.resize(count);
    for (uint32_t i = 0; i < count; i++) {
        tqs_plan *p = plans[i];
        if (!p) {
            delete B;
            return fail(TQS_E_ARG, "plan %u is NULL", i);
        }
        tqs_status st = check_noise(p, noises[i]);
        if (st) {
            delete B;
            return st;
        }
        if (p->prec != B->prec || p->reg_bits != B->reg_bits) {
            delete B;
            return fail(TQS_E_ARG, "plan %u: a batch needs one precision and one tile width", i);
        }
        BatchItem &it = B->items[i];
        it.p = p;
        it.nz = noises[i];
        build_meta(p, it.nz, &it.hm);
        Layout Ly0 = make_layout(p, it.nz->ev_gate.size(), p->n_leaves, 0);
        build_schedule(p, 0, p->arity[0], &it.tasks, &it.sched, Ly0.slot_base,
                       p->tune.no_merge ? nullptr : &it.hm);
        it.Ly = make_layout(p, it.nz->ev_gate.size(), p->n_leaves, it.sched.size(), states, 0);
        states = align256(states + (uint64_t)it.Ly.slots_total * it.Ly.state_bytes);
        it.leaf_base = B->leaves;
        B->leaves += p->n_leaves;
        const uint32_t L = (uint32_t)p->arity.size();
        for (uint32_t ti = 0; ti < it.tasks.size(); ti++) {
            const Task &t = it.tasks[ti];
            const tqs::Level &lv = p->levels[t.level];
            for (uint32_t k = 0; k < lv.pass_count; k++) it.ops.push_back({0, ti, lv.pass_begin + k, k == 0 ? 1u : 0u});
            if (t.level == L - 1) it.ops.push_back({1, ti, 0, 0});
        }
        B->steps = std::max<uint32_t>(B->steps, (uint32_t)it.ops.size());
    }
    // metadata regions after all states, then the segment tables
    uint64_t o = states;
    for (BatchItem &it : B->items) {
        it.Ly = make_layout(it.p, it.nz->ev_gate.size(), it.p->n_leaves, it.sched.size(), it.Ly.off_states, o);
        o = it.Ly.total;
    }
    B->npass.assign(B->steps, 0);
    B->nsamp.assign(B->steps, 0);
    for (BatchItem &it : B->items)
        for (uint32_t k = 0; k < it.ops.size(); k++) (it.ops[k].kind == 0 ? B->npass : B->nsamp)[k]++;
    const uint64_t pa = B->prec == TQS_C64 ? sizeof(PassArgs<float>) : sizeof(PassArgs<double>);
    const uint64_t sa = B->prec == TQS_C64 ? sizeof(SampleArgs<float>) : sizeof(SampleArgs<double>);
    B->table_at = align256(o);
    B->table_bytes = 0;
    for (uint32_t k = 0; k < B->steps; k++)
        B->table_bytes += align256(B->npass[k] * pa) + align256(B->nsamp[k] * sa);
    B->total = B->table_at + B->table_bytes;
    *out = B;
    return TQS_OK;
    TQS_GUARD_END
}

extern "C" tqs_status tqs_batch_info(const tqs_batch *b, uint64_t *workspace_bytes, uint64_t *leaves,
                                     uint32_t *steps) {
    if (!b) return fail(TQS_E_ARG, "batch is NULL");
    if (workspace_bytes) *workspace_bytes = b->total;
    if (leaves) *leaves = b->leaves;
    if (steps) *steps = b->steps;
    return TQS_OK;
}

extern "C" tqs_status tqs_batch_run(tqs_batch *b, void *d_workspace, uint64_t ws_bytes, void *stream,
                                    uint64_t *outcomes, tqs_run_stats *stats) {
    TQS_GUARD_BEGIN
    if (!b) return fail(TQS_E_ARG, "batch is NULL");
    if (b->prec == TQS_C64)
        return batch_run_t<float>(b, (unsigned char *)d_workspace, ws_bytes, (hipStream_t)stream, outcomes, stats);
    return batch_run_t<double>(b, (unsigned char *)d_workspace, ws_bytes, (hipStream_t)stream, outcomes, stats);
    TQS_GUARD_END
}

extern "C" tqs_status tqs_batch_use_graph(tqs_batch *b, uint32_t on) {
    if (!b) return fail(TQS_E_ARG, "batch is NULL");
    b->use_graph = on != 0;
    return TQS_OK;
}

extern "C" void tqs_batch_destroy(tqs_batch *b) {
    if (!b) return;
    for (void *e : b->events) (void)hipEventDestroy((hipEvent_t)e);
    if (b->graph_exec) (void)hipGraphExecDestroy((hipGraphExec_t)b->graph_exec);
    if (b->capture_stream) (void)hipStreamDestroy((hipStream_t)b->capture_stream);
    delete b;
}
