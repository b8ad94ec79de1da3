// Plan-specialised pass kernels: for every pass of a plan, HIP source in
// which the pass's ops are fixed (kinds, qubit roles and positions, phase
// terms as literals), compiled once per plan with hipRTC for the device the
// run uses and kept with the plan.  Same tile, same arithmetic per op as the
// generic pass kernel (pass_kernel.h); the device building blocks are in
// pass_jit.h.
//
// The specialised kernels read the trajectory's frame and events like the
// generic one, with two limits that keep them branch-free: at most three
// events strictly inside a phase run, and no X-frame change on register
// qubits between a run's register-only gates (their table is read at one
// frame).  jit_eligible() tells the executor which nodes a pass's
// specialised kernel can take; the others go to the generic kernel.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <algorithm>
#include <cmath>
#include <cinttypes>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "tqs_internal.h"

namespace tqs {

#include "jit_headers.inc"  // kJitHeaderCount, kJitHeaderNames[], kJitHeaderSrc[]: device headers as text

namespace {

void appendf(std::string &s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    const int n = std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (n < 0) return;
    if ((size_t)n < sizeof buf) {
        s.append(buf, (size_t)n);
        return;
    }
    std::string big((size_t)n + 1, '\0');
    va_start(ap, fmt);
    std::vsnprintf(&big[0], big.size(), fmt, ap);
    va_end(ap);
    big.resize((size_t)n);
    s += big;
}

// A phase as a literal of the accumulator width.
std::string lit(bool c64, uint64_t t) {
    char b[40];
    if (c64) std::snprintf(b, sizeof b, "0x%08" PRIx32 "u", (uint32_t)t);
    else std::snprintf(b, sizeof b, "0x%016" PRIx64 "ull", t);
    return b;
}

const char *role_name(uint32_t r) {
    switch (r) {
        case ROLE_LANE: return "ROLE_LANE";
        case ROLE_REG: return "ROLE_REG";
        case ROLE_FIXED: return "ROLE_FIXED";
        default: return "tqs::jit::kNone";
    }
}

// Register offset (in amplitudes) of register index j.
uint64_t reg_off(const PassDesc &d, uint32_t j) {
    uint64_t o = 0;
    for (uint32_t i = 0; i < d.nr; i++)
        if ((j >> i) & 1u) o |= 1ull << d.rq[i];
    return o;
}

// Register-only gates of a phase run: relative index of the first and last
// one (first > last: none).
void ro_span(const tqs_plan *p, const OpDesc &o, uint32_t *first, uint32_t *last) {
    *first = 1u;
    *last = 0u;
    bool any = false;
    for (uint32_t k = 0; k < o.ngates; k++) {
        const DiagGate &g = p->dgates[o.gates + k];
        const bool ro = g.role[0] == ROLE_REG && (g.nq == 1 || g.role[1] == ROLE_REG);
        if (!ro) continue;
        if (!any) *first = k;
        *last = k;
        any = true;
    }
}

void emit_diag(std::string &s, const tqs_plan *p, const PassDesc &d, const OpDesc &o, bool c64,
               uint32_t &table_slot) {
    const uint32_t nterm = [&] {
        uint32_t n = o.n_fix + o.n_lane;
        for (uint32_t b = 0; b < kMaxRegBits; b++) n += o.n_fixreg[b] + o.n_lanereg[b];
        return n;
    }();
    appendf(s, "  advance(w, KEY | %uu);\n  {\n", (unsigned)o.slot0);
    appendf(s, "    const RunFrames rf = run_frames(w, KEY | %uu, KEY | %uu);\n", (unsigned)o.slot0,
            (unsigned)o.slot1);
    // which accumulators the terms can touch
    bool cl[6] = {false}, cll[6][6] = {{false}}, cr[kMaxRegBits] = {false}, clr[6][kMaxRegBits] = {{false}};
    for (uint32_t t = 0; t < nterm; t++) {
        const DiagTerm &tm = p->terms[o.terms + t];
        if (tm.role[0] == ROLE_LANE) {
            cl[tm.pos[0]] = true;
            if (tm.nq == 2 && tm.role[1] == ROLE_LANE) {
                cl[tm.pos[1]] = true;
                cll[std::min(tm.pos[0], tm.pos[1])][std::max(tm.pos[0], tm.pos[1])] = true;
            }
            if (tm.nq == 2 && tm.role[1] == ROLE_REG) {
                cr[tm.pos[1]] = true;
                clr[tm.pos[0]][tm.pos[1]] = true;
            }
        } else if (tm.nq == 2 && tm.role[1] == ROLE_REG) {
            cr[tm.pos[1]] = true;
        }
    }
    if (nterm) {
        s += "    A c0 = 0;\n";
        for (int a = 0; a < 6; a++) {
            if (cl[a]) appendf(s, "    A cl%d = 0;\n", a);
            for (int b = a + 1; b < 6; b++)
                if (cll[a][b]) appendf(s, "    A cll%d_%d = 0;\n", a, b);
        }
        for (uint32_t i = 0; i < d.nr; i++) {
            if (cr[i]) appendf(s, "    A cr%u = 0;\n", i);
            for (int a = 0; a < 6; a++)
                if (clr[a][i]) appendf(s, "    A clr%d_%u = 0;\n", a, i);
        }
    }
    for (uint32_t t = 0; t < nterm; t++) {
        const DiagTerm &tm = p->terms[o.terms + t];
        const std::string T0 = lit(c64, tm.th[0]), T1 = lit(c64, tm.th[1]), T2 = lit(c64, tm.th[2]),
                          T3 = lit(c64, tm.th[3]);
        appendf(s, "    { const uint32_t f = rf.at(%uu);\n", (unsigned)tm.k);
        if (tm.nq == 1) {
            if (tm.role[0] == ROLE_LANE) {
                appendf(s,
                        "      const bool fu = ((f >> %u) & 1u) != 0; const A u0 = fu ? %s : %s, u1 = fu ? %s : %s;\n"
                        "      c0 += u0; cl%u += (A)(u1 - u0); }\n",
                        tm.phys[0], T1.c_str(), T0.c_str(), T0.c_str(), T1.c_str(), tm.pos[0]);
            } else {
                appendf(s, "      c0 += (((w.base ^ f) >> %u) & 1u) ? %s : %s; }\n", tm.phys[0], T1.c_str(),
                        T0.c_str());
            }
            continue;
        }
        if (tm.role[0] == ROLE_FIXED && tm.role[1] == ROLE_FIXED) {
            appendf(s,
                    "      const uint32_t y0 = ((w.base ^ f) >> %u) & 1u, y1 = ((w.base ^ f) >> %u) & 1u;\n"
                    "      c0 += y1 ? (y0 ? %s : %s) : (y0 ? %s : %s); }\n",
                    tm.phys[0], tm.phys[1], T3.c_str(), T2.c_str(), T1.c_str(), T0.c_str());
            continue;
        }
        appendf(s, "      const Ml<A> m = multilinear<A>(%s, %s, %s, %s, (f >> %u) & 1u, (f >> %u) & 1u);\n",
                T0.c_str(), T1.c_str(), T2.c_str(), T3.c_str(), tm.phys[0], tm.phys[1]);
        if (tm.role[0] == ROLE_LANE && tm.role[1] == ROLE_LANE) {
            const int a = tm.pos[0], b = tm.pos[1];
            appendf(s, "      c0 += m.a; cl%d += m.b; cl%d += m.g; cll%d_%d += m.d; }\n", a, b, std::min(a, b),
                    std::max(a, b));
        } else if (tm.role[0] == ROLE_LANE && tm.role[1] == ROLE_FIXED) {
            appendf(s,
                    "      const bool xw = ((w.base >> %u) & 1u) != 0;\n"
                    "      c0 += m.a + (xw ? m.g : (A)0); cl%u += m.b + (xw ? m.d : (A)0); }\n",
                    tm.phys[1], tm.pos[0]);
        } else if (tm.role[0] == ROLE_LANE && tm.role[1] == ROLE_REG) {
            appendf(s, "      c0 += m.a; cl%u += m.b; cr%u += m.g; clr%u_%u += m.d; }\n", tm.pos[0], tm.pos[1],
                    tm.pos[0], tm.pos[1]);
        } else {
            // fixed qubit 0, register qubit 1
            appendf(s,
                    "      const bool xu = ((w.base >> %u) & 1u) != 0;\n"
                    "      c0 += m.a + (xu ? m.b : (A)0); cr%u += m.g + (xu ? m.d : (A)0); }\n",
                    tm.phys[0], tm.pos[1]);
        }
    }
    uint32_t lm = 0;
    if (nterm) {
        s += "    const A C = c0";
        for (int a = 0; a < 6; a++)
            if (cl[a]) appendf(s, " + masked(cl%d, lb.m[%d])", a, a);
        for (int a = 0; a < 6; a++)
            for (int b = a + 1; b < 6; b++)
                if (cll[a][b]) appendf(s, " + masked(cll%d_%d, lb.m[%d] & lb.m[%d])", a, b, a, b);
        s += ";\n";
        // C is zero in every lane when its scalar coefficients all are
        s += "    const bool cz = uni((uint32_t)((c0";
        for (int a = 0; a < 6; a++)
            if (cl[a]) appendf(s, " | cl%d", a);
        for (int a = 0; a < 6; a++)
            for (int b = a + 1; b < 6; b++)
                if (cll[a][b]) appendf(s, " | cll%d_%d", a, b);
        s += ") == 0)) != 0u;\n    A lam[RB];\n";
        for (uint32_t i = 0; i < d.nr; i++) {
            if (!cr[i]) {
                appendf(s, "    lam[%u] = 0;\n", i);
                continue;
            }
            lm |= 1u << i;
            appendf(s, "    lam[%u] = cr%u", i, i);
            for (int a = 0; a < 6; a++)
                if (clr[a][i]) appendf(s, " + masked(clr%d_%u, lb.m[%d])", a, i, a);
            s += ";\n";
        }
        appendf(s, "    run_phase<R, RB, %uu>(v, C, lam, cz);\n", lm);
    }
    if (o.has_t) {
        uint32_t kf = 0, kl = 0;
        ro_span(p, o, &kf, &kl);
        appendf(s, "    { const uint32_t f = rf.at(%uu); const uint32_t fr = 0", kf);
        for (uint32_t i = 0; i < d.nr; i++) appendf(s, " | (((f >> %u) & 1u) << %u)", d.rq[i], i);
        // the plan's table at index j ^ fr, or the node's own table (frames
        // applied, every entry used) at index j
        appendf(s,
                ";\n      apply_table<R, RB>(v, ft ? ft + %uu : mats + %u, ft ? 0u : fr, ft ? 0xFFFFFFFFu : 0x%08xu); }\n",
                table_slot << d.nr, o.mat, o.tmask);
        table_slot++;
    }
    s += "  }\n";
}

// A one-qubit gate whose entries are all +-s (real, equal magnitudes): the
// sign pattern (bit 2r + c set where entry (r, c) is negative) and s; -1
// for any other op.
int butterfly(const tqs_plan *p, const OpDesc &o, double *s) {
    if (o.kind != OP_DENSE1 || o.nq != 1 || !o.real) return -1;
    const cd *m = p->mats.data() + o.mat;
    const double a = std::fabs(m[0].real());
    if (!(a > 0.0)) return -1;
    int neg = 0;
    for (int e = 0; e < 4; e++) {
        if (m[e].imag() != 0.0 || std::fabs(m[e].real()) != a) return -1;
        if (m[e].real() < 0.0) neg |= 1 << e;
    }
    *s = a;
    return neg;
}

// Lane bits an op mixes (dense ops whose target, or either qubit of a 4x4,
// is a lane qubit); a deferred per-lane sign on such a bit must be applied
// first.
uint32_t lane_bits_mixed(const OpDesc &o) {
    if (o.kind == OP_DIAGRUN) return 0;
    if (o.kind == OP_DENSE1) {
        const uint32_t tq = o.nq == 2 ? o.tq : 0u;
        return o.role[tq] == ROLE_LANE ? 1u << o.pos[tq] : 0u;
    }
    uint32_t m = 0;
    for (uint32_t q = 0; q < 2; q++)
        if (o.role[q] == ROLE_LANE) m |= 1u << o.pos[q];
    return m;
}

// sign_bits: lane bits the deferred per-lane sign depends on (updated).
void emit_dense(std::string &s, const tqs_plan *p, const OpDesc &o, double *scale, uint32_t *sign_bits) {
    if (lane_bits_mixed(o) & *sign_bits) {
        s += "  flush_sign<R, RB>(v, sg);\n";
        *sign_bits = 0;
    }
    appendf(s, "  advance(w, KEY | %uu);\n", (unsigned)o.slot0);
    appendf(s,
            "  { const uint32_t xl = local2(w.fx, %u, %u, %u), zl = local2(w.fz, %u, %u, %u);\n",
            o.phys[0], o.phys[1], o.nq, o.phys[0], o.phys[1], o.nq);
    double bs = 0.0;
    const int neg = butterfly(p, o, &bs);
    if (neg >= 0) {
        // its common factor joins the pass's scale
        *scale *= bs;
        if (o.role[0] == ROLE_LANE) {
            appendf(s, "    bf_lane<R, RB, %u, %d>(v, xl, zl, w, sg); }\n", (unsigned)o.pos[0], neg);
            *sign_bits |= 1u << o.pos[0];
        } else {
            appendf(s, "    bf_reg<R, RB, %u, %d>(v, xl, zl); }\n", (unsigned)o.pos[0], neg);
        }
        return;
    }
    if (o.kind == OP_DENSE1) {
        const uint32_t tq = o.nq == 2 ? o.tq : 0u, cq = 1u - tq;
        const uint32_t crole = o.nq == 2 ? o.role[cq] : 3u;
        const uint32_t cpos = o.nq == 2 ? o.pos[cq] : 0u;
        appendf(s, "    d1<R, RB, %s, %s, %u, %s, %u, %u, %u>(v, mats + %u, xl, zl, w); }\n",
                o.real ? "true" : "false", role_name(o.role[tq]), (unsigned)o.pos[tq], role_name(crole), cpos,
                (unsigned)o.nq, tq, o.mat);
    } else {
        const bool r0 = o.role[0] == ROLE_REG, r1 = o.role[1] == ROLE_REG;
        const bool sw = (r0 && r1) ? o.pos[0] > o.pos[1] : (!r0 && r1);
        const uint32_t p0 = sw ? o.pos[1] : o.pos[0], p1 = sw ? o.pos[0] : o.pos[1];
        const bool n0 = sw ? r1 : r0, n1 = sw ? r0 : r1;
        appendf(s, "    d2<R, RB, %s, %s, %s, %u, %u>(v, mats + %u, xl, zl, w); }\n", sw ? "true" : "false",
                n0 ? "true" : "false", n1 ? "true" : "false", p0, p1, o.mat);
    }
}

// The tile's origin w.base from the tile index expression `tile`.
void emit_base(std::string &s, const PassDesc &d, const char *tile) {
    s += "  w.base = 0";
    for (uint32_t i = 0; i < d.nfree; i++) appendf(s, " | (((%s >> %u) & 1u) << %u)", tile, i, d.fbits[i]);
    s += ";\n";
}

// Load the tile into v from the source state in HBM (or make |0..0>).
void emit_load(std::string &s, const PassDesc &d) {
    const bool full = d.nl == kLaneBits;
    const uint32_t nj = 1u << d.nr;
    s += "  cplx<R> v[1 << RB];\n";
    if (!full) appendf(s, "  const bool lane_ok = w.L < %uu;\n", 1u << d.nl);
    s += "  { const gptr<const cplx<R>> src = (gptr<const cplx<R>>)(a.states + (uint64_t)(init ? 0u : src_s) * "
         "a.slot_amps + w.base);\n";
    s += "  if (init) {\n";
    for (uint32_t j = 0; j < nj; j++)
        appendf(s, "    v[%u] = cplx<R>{%s, R(0)};\n", j, j == 0 ? "(w.base | w.L) == 0 ? R(1) : R(0)" : "R(0)");
    s += "  } else {\n";
    for (uint32_t j = 0; j < nj; j++) {
        if (full) appendf(s, "    v[%u] = src[%lluull + w.L];\n", j, (unsigned long long)reg_off(d, j));
        else
            appendf(s, "    v[%u] = lane_ok ? src[%lluull + w.L] : cplx<R>{R(0), R(0)};\n", j,
                    (unsigned long long)reg_off(d, j));
    }
    s += "  } }\n";
}

// The wave's frame and event cursor at the start of its node's level.
void emit_frame_init(std::string &s) {
    s += "  const uint32_t node = kconst(a.node_ids)[traj];\n"
         "  w.fx = uni(kconst(a.meta.frame0)[2 * node]);\n"
         "  w.fz = uni(kconst(a.meta.frame0)[2 * node + 1]);\n"
         "  w.e = uni(kconst(a.meta.ev_off)[node]);\n"
         "  w.e1 = uni(kconst(a.meta.ev_off)[node + 1]);\n"
         "  w.pos = kconst(a.meta.ev_pos);\n  w.dx = kconst(a.meta.ev_dx);\n  w.dz = kconst(a.meta.ev_dz);\n"
         "  w.nxt = w.e < w.e1 ? uni(w.pos[w.e]) : 0xFFFFFFFFu;\n"
         "  const kptr<cplx<R>> mats = kconst(a.mats);\n"
         "  const LaneBits lb = lane_bits(w.L);\n"
         "  (void)lb;\n";
}

// The pass's ops on v (frame tables, fused blocks, phase runs, dense ops),
// then the butterflies' common factor.
void emit_ops(std::string &s, const tqs_plan *p, uint32_t pi) {
    const PassDesc &d = p->passes[pi];
    const bool c64 = p->prec == TQS_C64;
    if (jit_table_entries(p, pi)) {
        // the node's own frame tables for this pass, if it has them
        appendf(s,
                "  kptr<cplx<R>> ft = nullptr;\n"
                "  { const uint32_t co = uni(kconst(a.meta.ct_off)[node]);\n"
                "    if (co != 0xFFFFFFFFu) {\n"
                "      const kptr<uint32_t> dir = kconst(a.meta.ct_dir);\n"
                "      const uint32_t cnt = uni(dir[co]);\n"
                "      for (uint32_t i = 0; i < cnt; i++)\n"
                "        if (uni(dir[co + 1 + 2 * i]) == %uu) ft = kconst((const cplx<R> *)a.meta.ctab) + uni(dir[co + 2 + 2 * i]);\n"
                "    } }\n",
                pi);
    }
    uint32_t table_slot = 0;
    double scale = 1.0;      // product of the butterflies' common factors
    uint32_t sign_bits = 0;  // lane bits of the deferred per-lane sign
    bool lane_bf = false;
    for (uint32_t oi = d.op_begin; oi < d.op_begin + d.op_count; oi++) {
        double bs = 0.0;
        if (butterfly(p, p->ops[oi], &bs) >= 0 && p->ops[oi].role[0] == ROLE_LANE) lane_bf = true;
    }
    if (lane_bf) s += "  R sg = R(1);  // deferred per-lane sign of the lane butterflies\n";
    size_t bi = 0;
    while (bi < p->blocks.size() && p->blocks[bi].pass < pi) bi++;
    for (uint32_t oi = d.op_begin; oi < d.op_begin + d.op_count; oi++) {
        const OpDesc &o = p->ops[oi];
        if (bi < p->blocks.size() && p->blocks[bi].pass == pi && p->blocks[bi].op_begin == oi) {
            // a fused register-only run on the matrix cores; the frame's
            // register bits conjugate it
            const FusedBlock &fb = p->blocks[bi++];
            appendf(s, "  advance(w, KEY | %uu);\n  { const uint32_t xr = 0", (unsigned)o.slot0);
            for (uint32_t i = 0; i < d.nr; i++) appendf(s, " | (((w.fx >> %u) & 1u) << %u)", d.rq[i], i);
            s += ", zr = 0";
            for (uint32_t i = 0; i < d.nr; i++) appendf(s, " | (((w.fz >> %u) & 1u) << %u)", d.rq[i], i);
            appendf(s, ";\n    mfma32(v, mats + %u, xr, zr, w.L); }\n", fb.mat);
            oi = fb.op_end - 1;
            continue;
        }
        if (o.kind == OP_DIAGRUN) emit_diag(s, p, d, o, c64, table_slot);
        else emit_dense(s, p, o, &scale, &sign_bits);
    }
    if (sign_bits) appendf(s, "  scale_tile<R, RB>(v, R(%.17g) * sg);\n", scale);
    else if (scale != 1.0) appendf(s, "  scale_tile<R, RB>(v, R(%.17g));\n", scale);
}

// Store v to the node's state in HBM, with the sampling partials when the
// pass is the leaf level's last.
void emit_store(std::string &s, const PassDesc &d, const char *tile) {
    const bool full = d.nl == kLaneBits;
    const uint32_t nj = 1u << d.nr;
    s += "  { const gptr<cplx<R>> dst = (gptr<cplx<R>>)(a.states + (uint64_t)dst_s * a.slot_amps + w.base);\n";
    for (uint32_t j = 0; j < nj; j++) {
        if (full) appendf(s, "  dst[%lluull + w.L] = v[%u];\n", (unsigned long long)reg_off(d, j), j);
        else appendf(s, "  if (lane_ok) dst[%lluull + w.L] = v[%u];\n", (unsigned long long)reg_off(d, j), j);
    }
    s += "  }\n";
    if (full) appendf(s, "  if (a.part) tile_partials<R, RB>(v, a, traj, %s, %uu, w.L);\n", tile, (unsigned)d.nfree);
}

void emit_header(std::string &s, const tqs_plan *p) {
    const bool c64 = p->prec == TQS_C64;
    appendf(s, "  using namespace tqs;\n  using namespace tqs::jit;\n  using R = %s;\n  using A = %s;\n",
            c64 ? "float" : "double", c64 ? "uint32_t" : "uint64_t");
}

// One pass over a chunk of states: one wave per tile of one state.
void emit_pass(std::string &s, const tqs_plan *p, uint32_t pi) {
    const PassDesc &d = p->passes[pi];
    const bool c64 = p->prec == TQS_C64;
    const int waves = (c64 && d.nr <= 5) ? 3 : 1;
    appendf(s, "extern \"C\" __global__ __launch_bounds__(64, %d) void tqs_jit_p%u(tqs::PassLaunch<%s> pl) {\n",
            waves, pi, c64 ? "float" : "double");
    emit_header(s, p);
    appendf(s, "  constexpr int RB = %u;\n  constexpr uint32_t KEY = %uu << 16;\n", (unsigned)d.nr, pi);
    s += "  const uint32_t nwg = gridDim.x, bid = blockIdx.x;\n"
         "  const uint32_t wall = (bid & 7u) * (nwg >> 3) + (bid >> 3);\n"
         "  const PassArgs<R> &a = pl.one;\n"
         "  if (wall >= a.work) return;\n"
         "  const uint32_t ti = wall % a.count, tile = wall / a.count;\n"
         "  const uint32_t traj = a.perm ? kconst(a.perm)[ti] : ti;\n"
         "  Wave w;\n  w.L = threadIdx.x;\n";
    emit_base(s, d, "tile");
    s += "  const uint32_t src_s = kconst(a.src_slot)[traj], dst_s = kconst(a.dst_slot)[traj];\n"
         "  const bool init = src_s == kInit;\n";
    emit_load(s, d);
    emit_frame_init(s);
    if (pi > 0) s += "  advance(w, KEY - 1u);\n";
    emit_ops(s, p, pi);
    emit_store(s, d, "tile");
    s += "}\n\n";
}

// Process-wide cache of compiled code objects by source text.
std::mutex g_cache_mu;
std::unordered_map<std::string, std::vector<char>> g_cache;

}  // namespace

bool jit_pass_supported(const tqs_plan *p, uint32_t pi) {
    const PassDesc &d = p->passes[pi];
    return d.nr >= 1 && d.op_count > 0;
}

std::string jit_source(const tqs_plan *p) {
    std::string s;
    s += "// plan-specialised pass kernels (generated)\n"
         "typedef __hip_internal::uint8_t uint8_t;\n"
         "typedef __hip_internal::uint16_t uint16_t;\n"
         "typedef __hip_internal::uint32_t uint32_t;\n"
         "typedef __hip_internal::uint64_t uint64_t;\n"
         "typedef __hip_internal::int32_t int32_t;\n"
         "typedef __hip_internal::int64_t int64_t;\n"
         "#include \"pass_jit.h\"\n"
         "namespace tqs { namespace jit {\n"
         "template <typename T> using gptr = __attribute__((address_space(1))) T *;\n"
         "} }\n\n";
    for (uint32_t pi = 0; pi < (uint32_t)p->passes.size(); pi++)
        if (jit_pass_supported(p, pi)) emit_pass(s, p, pi);
    return s;
}

// Compile the plan's kernels (or take them from the cache); no device needed.
tqs_status jit_compile(tqs_plan *p) {
    if (!p->jit_code.empty()) return TQS_OK;
    const std::string src = jit_source(p);
    {
        std::lock_guard<std::mutex> lock(g_cache_mu);
        auto it = g_cache.find(src);
        if (it != g_cache.end()) {
            p->jit_code = it->second;
            return TQS_OK;
        }
    }
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "tqs_jit.hip", kJitHeaderCount, kJitHeaderSrc, kJitHeaderNames) !=
        HIPRTC_SUCCESS)
        return fail(TQS_E_HIP, "hiprtcCreateProgram failed");
    const char *opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17",
                          // no packed FP32 instructions in generated code
                          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                          "-mllvm", "-simplifycfg-sink-common=false"};
    const hiprtcResult rc = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof opts[0]), opts);
    if (rc != HIPRTC_SUCCESS) {
        size_t ls = 0;
        hiprtcGetProgramLogSize(prog, &ls);
        std::string log(ls, '\0');
        if (ls) hiprtcGetProgramLog(prog, &log[0]);
        hiprtcDestroyProgram(&prog);
        return fail(TQS_E_HIP, "hipRTC compile of the plan's pass kernels failed: %.600s", log.c_str());
    }
    size_t cs = 0;
    hiprtcGetCodeSize(prog, &cs);
    std::vector<char> code(cs);
    hiprtcGetCode(prog, code.data());
    hiprtcDestroyProgram(&prog);
    p->jit_code = code;
    std::lock_guard<std::mutex> lock(g_cache_mu);
    g_cache.emplace(src, std::move(code));
    return TQS_OK;
}

// Compile if needed and load the kernels on the current device.
tqs_status jit_prepare(tqs_plan *p) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return fail(TQS_E_HIP, "hipGetDevice failed");
    if (p->jit_module && p->jit_device == dev) return TQS_OK;
    jit_release(p);
    tqs_status st = jit_compile(p);
    if (st) return st;
    hipModule_t mod = nullptr;
    if (hipModuleLoadData(&mod, p->jit_code.data()) != hipSuccess)
        return fail(TQS_E_HIP, "hipModuleLoadData of the plan's pass kernels failed");
    p->jit_fn.assign(p->passes.size(), nullptr);
    for (uint32_t pi = 0; pi < (uint32_t)p->passes.size(); pi++) {
        if (!jit_pass_supported(p, pi)) continue;
        char name[32];
        std::snprintf(name, sizeof name, "tqs_jit_p%u", pi);
        hipFunction_t fn = nullptr;
        if (hipModuleGetFunction(&fn, mod, name) != hipSuccess) {
            (void)hipModuleUnload(mod);
            p->jit_fn.clear();
            return fail(TQS_E_HIP, "kernel %s missing from the compiled module", name);
        }
        p->jit_fn[pi] = (void *)fn;
    }
    p->jit_module = (void *)mod;
    p->jit_device = dev;
    return TQS_OK;
}

void jit_release(tqs_plan *p) {
    if (p->jit_module) (void)hipModuleUnload((hipModule_t)p->jit_module);
    p->jit_module = nullptr;
    p->jit_fn.clear();
    p->jit_device = -1;
}

// Per pass, the phase runs' slots and register-only spans (for routing).
void jit_runs(const tqs_plan *p, std::vector<std::vector<JitRun>> *runs,
              std::vector<std::vector<JitBlock>> *blocks) {
    runs->assign(p->passes.size(), {});
    blocks->assign(p->passes.size(), {});
    for (const FusedBlock &fb : p->blocks) {
        JitBlock b;
        b.first = (fb.pass << 16) | p->ops[fb.op_begin].slot0;
        b.last = (fb.pass << 16) | p->ops[fb.op_end - 1].slot0;
        (*blocks)[fb.pass].push_back(b);
    }
    for (uint32_t pi = 0; pi < (uint32_t)p->passes.size(); pi++) {
        const PassDesc &d = p->passes[pi];
        uint32_t regmask = 0;
        for (uint32_t i = 0; i < d.nr; i++) regmask |= 1u << d.rq[i];
        for (uint32_t oi = d.op_begin; oi < d.op_begin + d.op_count; oi++) {
            const OpDesc &o = p->ops[oi];
            if (o.kind != OP_DIAGRUN) continue;
            JitRun r;
            r.s0 = o.slot0;
            r.s1 = o.slot1;
            r.ngates = o.ngates;
            r.ro_first = 1;
            r.ro_last = 0;
            if (o.has_t) ro_span(p, o, &r.ro_first, &r.ro_last);
            r.regmask = regmask;
            r.op = oi;
            (*runs)[pi].push_back(r);
        }
    }
}

// How the specialised kernel of pass pi takes a node whose events (sorted
// keys pos[0..n), X masks dx) are given: not at all (an event between the
// ops of a fused block, or more than three inside a run), with its own frame tables (an X change on register qubits
// between a run's register-only gates), or as is.
JitFit jit_fit(const std::vector<JitRun> &runs, const std::vector<JitBlock> &blocks, uint32_t pi,
              const uint32_t *pos, const uint32_t *dx, uint32_t n) {
    const uint32_t key = pi << 16;
    bool tables = false;
    // an event between the ops of a fused block
    for (const JitBlock &b : blocks)
        for (uint32_t e = 0; e < n; e++)
            if (pos[e] > b.first && pos[e] <= b.last) return JIT_NO;
    for (const JitRun &r : runs) {
        uint32_t inside = 0;
        for (uint32_t e = 0; e < n; e++) {
            const uint32_t k = pos[e];
            if (k <= (key | r.s0) || k >= (key | r.s1)) continue;
            inside++;
            const uint32_t rel = (k & 0xFFFFu) - r.s0;
            if (r.ro_first <= r.ro_last && rel > r.ro_first && rel <= r.ro_last && (dx[e] & r.regmask)) tables = true;
        }
        if (inside > 3 || (inside && r.ngates >= 255)) return JIT_NO;
    }
    return tables ? JIT_TABLES : JIT_YES;
}

uint32_t jit_table_entries(const tqs_plan *p, uint32_t pi) {
    const PassDesc &d = p->passes[pi];
    uint32_t n = 0;
    for (uint32_t oi = d.op_begin; oi < d.op_begin + d.op_count; oi++)
        if (p->ops[oi].kind == OP_DIAGRUN && p->ops[oi].has_t) n += 1u << d.nr;
    return n;
}

void jit_frame_tables(const tqs_plan *p, uint32_t pi, uint32_t fx0, const uint32_t *pos, const uint32_t *dx,
                      uint32_t n, std::vector<cd> *out) {
    const PassDesc &d = p->passes[pi];
    const uint32_t nt = 1u << d.nr;
    for (uint32_t oi = d.op_begin; oi < d.op_begin + d.op_count; oi++) {
        const OpDesc &o = p->ops[oi];
        if (o.kind != OP_DIAGRUN || !o.has_t) continue;
        const size_t at = out->size();
        out->resize(at + nt, cd(1.0, 0.0));
        for (uint32_t k = 0; k < o.ngates; k++) {
            const DiagGate &g = p->dgates[o.gates + k];
            const bool ro = g.role[0] == ROLE_REG && (g.nq == 1 || g.role[1] == ROLE_REG);
            if (!ro) continue;
            // the X frame this gate sees: every event up to its slot
            const uint32_t gk = (pi << 16) | (o.slot0 + k);
            uint32_t f = fx0;
            for (uint32_t e = 0; e < n && pos[e] <= gk; e++) f ^= dx[e];
            uint32_t fr = 0;
            for (uint32_t i = 0; i < d.nr; i++) fr |= ((f >> d.rq[i]) & 1u) << i;
            for (uint32_t t = 0; t < nt; t++) {
                const uint32_t y = t ^ fr;
                uint32_t r = 0;
                for (uint32_t q = 0; q < g.nq; q++) r |= ((y >> g.pos[q]) & 1u) << q;
                // (plain complex product: std::complex's operator* goes through
                // a library call with infinity and NaN recovery)
                const cd a = (*out)[at + t], b = p->mats[g.d + r];
                (*out)[at + t] = cd(a.real() * b.real() - a.imag() * b.imag(), a.real() * b.imag() + a.imag() * b.real());
            }
        }
    }
}

}  // namespace tqs

extern "C" {

tqs_status tqs_plan_compile(tqs_plan *p) {
    if (!p) return tqs::fail(TQS_E_ARG, "plan is NULL");
    if (p->tune.jit != 1) return TQS_OK;
    try {
        return tqs::jit_compile(p);
    } catch (...) {
        return tqs::fail(TQS_E_OOM, "host allocation failed");
    }
}

tqs_status tqs_plan_jit_source(const tqs_plan *p, char *buf, uint64_t cap, uint64_t *len) {
    if (!p || !len) return tqs::fail(TQS_E_ARG, "plan or len is NULL");
    try {
        const std::string s = tqs::jit_source(p);
        *len = s.size() + 1;
        if (buf && cap) {
            const uint64_t n = std::min<uint64_t>(cap - 1, s.size());
            std::memcpy(buf, s.data(), n);
            buf[n] = '\0';
        }
        return TQS_OK;
    } catch (...) {
        return tqs::fail(TQS_E_OOM, "host allocation failed");
    }
}

}  // extern "C"
