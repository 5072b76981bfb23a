// Pass specialisation at run time: every fused pass becomes a straight-line
// kernel compiled with hipRTC for gfx950.
//
// The generic pass kernel interprets its op list: each op picks, at run time,
// the register pairs of its target slot, its control mode and its kind.  The
// amplitudes then flow through a many-way branch at every op, and the
// compiler answers with copies of the whole register set per op (more VALU
// work than the arithmetic itself for complex128) plus a chain of dependent
// scalar loads.  A pass kernel generated from the op list has none of this:
// register slots, register-bit layouts, in-tile control masks and op kinds
// are compile-time facts, so an exact NOT is a renaming of registers, a
// control on a register bit selects pairs at compile time, and the FP64 work
// is the 16 multiply-adds per amplitude pair and nothing else.  What changes
// between circuits of one shape stays run-time data read from the same
// descriptors as before: matrices, out-of-tile controls, the tile's global
// bits.  Kernels are cached by the signature of everything the generator
// reads from a pass.
#include <hip/hiprtc.h>

#include <algorithm>
#include <array>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "fused.h"

namespace {

// Device prelude of every generated kernel.  The descriptor structs repeat
// the host layout (FPass, FOp); their sizes are checked at compile time.
const char *kPrelude = R"PRELUDE(
typedef double c128 __attribute__((ext_vector_type(2)));
typedef float c64 __attribute__((ext_vector_type(2)));
typedef float v4f __attribute__((ext_vector_type(4)));
struct FOp { int kind; int lbit; unsigned lctrl; int slot; unsigned long long gctrl; unsigned long long gtbit; double m[8]; };
struct FPass { int k; int nlow; int first; int nops; signed char bits[16]; };
static_assert(sizeof(FOp) == 96, "FOp");
static_assert(sizeof(FPass) == 32, "FPass");
__device__ __forceinline__ unsigned long long ins0(unsigned long long t, int p) {
    const unsigned long long lo = t & ((1ull << p) - 1);
    return ((t & ~lo) << 1) | lo;
}
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}
)PRELUDE";

struct Gen {
    std::string s;
    void line(const char *fmt, ...) __attribute__((format(printf, 2, 3))) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        s += buf;
        s += '\n';
    }
};

// Register layout: rb[i] = local bit of register slot i.
struct Layout {
    int rb[4];
};

std::string deposit_expr(int K, int M, const Layout &L) {
    uint32_t rmask = 0;
    for (int i = 0; i < M; ++i) rmask |= 1u << L.rb[i];
    std::string e = "0u";
    int src = 0;
    char buf[96];
    for (int b = 0; b < K; ++b) {
        if ((rmask >> b) & 1) continue;
        snprintf(buf, sizeof buf, " | (((unsigned)t >> %d) & 1u) << %d", src, b);
        e += buf;
        ++src;
    }
    return e;
}

uint32_t reg_off(const Layout &L, int M, int j) {
    uint32_t x = 0;
    for (int i = 0; i < M; ++i)
        if ((j >> i) & 1) x |= 1u << L.rb[i];
    return x;
}

// Register-slot mask and thread-bit mask of a local control mask.
void split_ctrl(const Layout &L, int M, uint32_t lctrl, int &creg, uint32_t &cthr) {
    creg = 0;
    cthr = lctrl;
    for (int i = 0; i < M; ++i)
        if ((lctrl >> L.rb[i]) & 1) {
            creg |= 1 << i;
            cthr &= ~(1u << L.rb[i]);
        }
}

// A phase run: the OP_FACTOR terms ops[o..e) multiplied into one factor per
// register.  Terms on no register slot go into one per-lane product, terms
// on one slot into a per-slot product; the factor of register j is then the
// per-lane product times the per-slot products of j's set slots, built as a
// product tree over the slots that have any (2^s - 1 complex multiplies for
// s such slots), times the terms on two or more slots where j has them all.
// Each register then takes one complex multiply.
void phase_run(Gen &g, const FOp *ops, int o, int e, int M, bool c128) {
    const char *R = c128 ? "double" : "float";
    const int V = 1 << M;
    auto acc_name = [&](int x) {
        const uint32_t mask = uint32_t(ops[x].lbit) & 0xffu;
        char b[16];
        if (mask == 0)
            snprintf(b, sizeof b, "pg");
        else if (__builtin_popcount(mask) == 1)
            snprintf(b, sizeof b, "pr%d", __builtin_ctz(mask));
        else
            snprintf(b, sizeof b, "pc%d", x);
        return std::string(b);
    };
    auto mul = [&](const std::string &d, const std::string &a, const std::string &b, bool decl) {
        g.line("    %s%sr = %sr * %sr - %si * %si, %si = %sr * %si + %si * %sr;", decl ? "const " : "",
               decl ? (std::string(R) + " " + d).c_str() : d.c_str(), a.c_str(), b.c_str(), a.c_str(), b.c_str(),
               d.c_str(), a.c_str(), b.c_str(), a.c_str(), b.c_str());
    };
    g.line("    { // phase run");
    if (((ops[o].lbit >> 8) & 0xff) == 254) {
        // every factor known on the host: one table entry per register
        for (int j = 0; j < V; ++j) {
            g.line("    { const FOp &cur = op[%d]; const %s fr = (%s)cur.m[%d], fi = (%s)cur.m[%d];", o + j / 4, R, R,
                   2 * (j % 4), R, 2 * (j % 4) + 1);
            g.line("      const %s x0 = v[%d].x, x1 = v[%d].y; v[%d].x = fr * x0 - fi * x1; v[%d].y = fr * x1 + fi * x0; }", R,
                   j, j, j, j);
        }
        g.line("    } // phase run");
        return;
    }
    std::vector<std::string> names;
    std::unordered_set<std::string> declared;
    uint32_t B = 0;
    for (int x = o; x < e; ++x) {
        names.push_back(acc_name(x));
        if (declared.insert(names.back()).second) g.line("    %s %sr, %si;", R, names.back().c_str(), names.back().c_str());
        if (__builtin_popcount(uint32_t(ops[x].lbit) & 0xffu) >= 1) B |= uint32_t(ops[x].lbit) & 0xffu;
    }
    std::unordered_set<std::string> set;
    for (int x = o; x < e; ++x) {
        const FOp &f = ops[x];
        const int code = (f.lbit >> 8) & 0xff;
        const std::string &n = names[size_t(x - o)];
        g.line("    { const FOp &cur = op[%d];", x);
        if (code == 0) {
            g.line("    %s fr = (%s)cur.m[0], fi = (%s)cur.m[1];", R, R, R);
        } else {
            if (code == 255)
                g.line("    const bool hi = (base & cur.gtbit) != 0ull;");
            else
                g.line("    const bool hi = (tp >> %d) & 1u;", code - 1);
            g.line("    %s fr = hi ? (%s)cur.m[2] : (%s)cur.m[0], fi = hi ? (%s)cur.m[3] : (%s)cur.m[1];", R, R, R, R,
                   R);
        }
        std::string cond;
        if (f.lctrl) {
            char c[64];
            snprintf(c, sizeof c, "((tp & %uu) == %uu)", f.lctrl, f.lctrl);
            cond = c;
        }
        if (f.gctrl) cond += std::string(cond.empty() ? "" : " && ") + "((base & cur.gctrl) == cur.gctrl)";
        if (!cond.empty()) g.line("    if (!(%s)) { fr = 1; fi = 0; }", cond.c_str());
        if (set.insert(n).second) {
            g.line("    %sr = fr; %si = fi; }", n.c_str(), n.c_str());
        } else {
            g.line("    const %s tr = %sr * fr - %si * fi; %si = %sr * fi + %si * fr; %sr = tr; }", R, n.c_str(), n.c_str(),
                   n.c_str(), n.c_str(), n.c_str(), n.c_str());
        }
    }
    // factor of register j: entry j & B of the tree ("" = exactly one)
    std::vector<std::string> P(size_t(V), "");
    if (set.count("pg")) P[0] = "pg";
    int tmp = 0;
    auto fresh = [&]() {
        char b[16];
        snprintf(b, sizeof b, "pq%d", tmp++);
        return std::string(b);
    };
    for (int k = 0; k < M; ++k) {
        if (!((B >> k) & 1)) continue;
        char rk[16];
        snprintf(rk, sizeof rk, "pr%d", k);
        const bool has = set.count(rk) != 0;
        for (int j = 0; j < V; ++j) {
            if ((uint32_t(j) & ~B) || (j >> k)) continue;  // entries built so far: subsets of B below bit k
            const int jj = j | (1 << k);
            if (!has)
                P[size_t(jj)] = P[size_t(j)];
            else if (P[size_t(j)].empty())
                P[size_t(jj)] = rk;
            else {
                const std::string d = fresh();
                mul(d, P[size_t(j)], rk, true);
                P[size_t(jj)] = d;
            }
        }
    }
    for (int x = o; x < e; ++x) {
        const uint32_t mask = uint32_t(ops[x].lbit) & 0xffu;
        if (__builtin_popcount(mask) < 2) continue;
        const std::string &c = names[size_t(x - o)];
        for (int j = 0; j < V; ++j) {
            if ((uint32_t(j) & ~B) || (uint32_t(j) & mask) != mask) continue;
            if (P[size_t(j)].empty()) {
                P[size_t(j)] = c;
            } else {
                const std::string d = fresh();
                mul(d, P[size_t(j)], c, true);
                P[size_t(j)] = d;
            }
        }
    }
    for (int j = 0; j < V; ++j) {
        const std::string &p = P[size_t(uint32_t(j) & B)];
        if (p.empty()) continue;
        g.line("    { const %s x0 = v[%d].x, x1 = v[%d].y; v[%d].x = %sr * x0 - %si * x1; v[%d].y = %sr * x1 + %si * x0; }",
               R, j, j, j, p.c_str(), p.c_str(), j, p.c_str(), p.c_str());
    }
    g.line("    } // phase run");
}

// Generates the kernel of one pass.  ops: the pass's host descriptors.
std::string generate(int dtype, int K, int M, const FPass &TP, const FOp *ops, int nops, bool mfma_on, int waves) {
    const bool c128 = dtype == SV_C128;
    const char *T = c128 ? "c128" : "c64";
    const char *R = c128 ? "double" : "float";
    const int V = 1 << M, NT = 1 << (K - M), SB = c128 ? 4 : 5;
    // complex64 dense ops on the matrix cores (v_mfma_f32_4x4x1_16b, see
    // OP_DENSE below).  A lane's outputs read the A operand of the other
    // lanes of its group of four, so every group must be active: the tile
    // needs at least 4 threads.
    const bool mfma = !c128 && mfma_on && NT >= 4;
    bool any_remap = false, any_table = false;
    for (int o = 0; o < nops; ++o) {
        any_remap |= ops[o].kind == OP_REMAP;
        any_table |= (ops[o].kind == OP_DENSE || ops[o].kind == OP_DIAG) && ops[o].slot >= 0;
    }
    // tile bits as constants (a kernel per tile shape): every HBM index is
    // a per-thread part plus a constant per register.  Passes of trajectory
    // batches can keep them as run-time data instead and share one kernel
    // among tile shapes (batch_const_bits 0: 1.5% slower noisy Grover
    // batches with the matrix cores; plain passes 3-5% slower that way)
    const bool cbits = !any_table || svi_config().batch_const_bits != 0;

    Gen g;
    g.s = kPrelude;
    // waves > 0: registers budgeted for that many waves per SIMD (the
    // compiler otherwise sizes them for the occupancy the LDS tile allows)
    char occ[64] = "";
    if (waves > 0) snprintf(occ, sizeof occ, " __attribute__((amdgpu_waves_per_eu(%d)))", waves);
    g.line("extern \"C\" __global__ __launch_bounds__(%d)%s void sv_pass(%s *__restrict__ a, const FPass *__restrict__ pass,",
           NT, occ, T);
    g.line("        const FOp *__restrict__ ops, const %s *__restrict__ table, unsigned nslots, int tile_bits, int n) {", R);
    if (any_remap) g.line("    __shared__ %s lds[%d];", T, 1 << K);
    g.line("    const FPass P = *pass;");
    g.line("    const int t = threadIdx.x;");
    if (mfma) g.line("    const int ri = t & 3;  // row of a 4x4x1 MFMA block this lane feeds as A");
    if (!cbits) g.line("    const unsigned lowmask = (1u << P.nlow) - 1u;");
    // workgroup w: tile (w mod 2^tile_bits) of register (w >> tile_bits);
    // registers are stored back to back and own rows of nslots matrices
    g.line("    const unsigned long long reg = (unsigned long long)blockIdx.x >> tile_bits;");
    g.line("    a += reg << n;");
    g.line("    const %s *trow = table + reg * nslots * 8ull;", R);
    // the tile's index bits are compile-time facts of the kernel: tile bit i
    // sits at index bit gbit(i) (the lowest nlow contiguous)
    auto gbit = [&](int i) { return i < TP.nlow ? i : int(TP.bits[i]); };
    g.line("    unsigned long long base = (unsigned long long)blockIdx.x & ((1ull << tile_bits) - 1ull);");
    if (cbits) {
        for (int i = 0; i < K; ++i) g.line("    base = ins0(base, %d);", int(TP.bits[i]));
    } else {
        g.line("#pragma unroll");
        g.line("    for (int i = 0; i < %d; ++i) base = ins0(base, P.bits[i]);", K);
    }
    g.line("    const FOp *op = ops + P.first;");
    Layout L;
    for (int i = 0; i < M; ++i) L.rb[i] = K - M + i;
    g.line("    unsigned tp = %s;", deposit_expr(K, M, L).c_str());
    // index of register j: gth | gj[j] (constant tile bits) or deposited
    // from the descriptor (run-time tile bits)
    auto run_time_index = [&](const char *what) {
        g.line("#pragma unroll");
        g.line("    for (int j = 0; j < %d; ++j) {", V);
        g.line("        const unsigned r = tp | ((unsigned)j << %d);", K - M);
        g.line("        unsigned long long gi = base | (r & lowmask);");
        g.line("#pragma unroll");
        g.line("        for (int i = 0; i < %d; ++i)", K);
        g.line("            if (i >= P.nlow) gi |= (unsigned long long)((r >> i) & 1u) << P.bits[i];");
        g.line("        %s", what);
        g.line("    }");
    };
    if (cbits) {
        // thread part of the index (tile bits 0..K-M-1 from tp), once
        std::string e = "base";
        const int nl = std::min(TP.nlow, K - M);
        if (nl > 0) {
            char b[96];
            snprintf(b, sizeof b, " | (unsigned long long)(tp & %uu)", (1u << nl) - 1u);
            e += b;
        }
        for (int i = nl; i < K - M; ++i) {
            char b[96];
            snprintf(b, sizeof b, " | ((unsigned long long)((tp >> %d) & 1u) << %d)", i, gbit(i));
            e += b;
        }
        g.line("    const unsigned long long gth = %s;", e.c_str());
    }
    // register part of the index: a constant per register
    std::vector<unsigned long long> gj(size_t(V), 0ull);
    for (int j = 0; j < V; ++j)
        for (int i = K - M; i < K; ++i)
            if ((j >> (i - (K - M))) & 1) gj[size_t(j)] |= 1ull << gbit(i);
    g.line("    %s v[%d];", T, V);
    if (cbits) {
        for (int j = 0; j < V; ++j)
            g.line("    v[%d] = __builtin_nontemporal_load(a + (gth | %lluull));", j, gj[size_t(j)]);
    } else {
        run_time_index("v[j] = __builtin_nontemporal_load(a + gi);");
    }
    // the same map on a constant index
    auto swz_const = [&](uint32_t r) { return r ^ (((r >> SB) ^ (r >> (2 * SB))) & ((1u << SB) - 1u)); };
    auto swz = [&](const std::string &r) {
        char buf[256];
        snprintf(buf, sizeof buf, "((%s) ^ ((((%s) >> %d) ^ ((%s) >> %d)) & %du))", r.c_str(), r.c_str(), SB, r.c_str(),
                 2 * SB, (1u << SB) - 1);
        return std::string(buf);
    };
    bool lds_live = false;
    // Runs of consecutive diagonal ops commute.  Inside a run, a diagonal op
    // whose conditions involve no register bit scales every register with a
    // given target value by one per-lane factor: such ops are multiplied into
    // per-lane accumulators (one pair per target register slot, one for
    // targets on thread bits or outside the tile) and the accumulators are
    // applied once when the run ends.  A run of controlled phases with one
    // target (the QFT's) then costs one complex multiply per op and lane
    // plus one per register, instead of one per op and register.
    bool run_open = false;
    uint32_t run_g1 = 0, run_g0 = 0;  // slots with a used accumulator
    bool run_all = false;
    auto close_run = [&]() {
        if (!run_open) return;
        auto apply = [&](int j, const char *gr, const char *gi) {
            g.line("    { const %s x = v[%d]; v[%d].x = %s * x.x - %s * x.y; v[%d].y = %s * x.y + %s * x.x; }", T, j, j,
                   gr, gi, j, gr, gi);
        };
        for (int sl = 0; sl < M; ++sl)
            for (int j = 0; j < V; ++j) {
                char gr[16], gi[16];
                const bool hi = (j >> sl) & 1;
                if (hi && ((run_g1 >> sl) & 1)) {
                    snprintf(gr, sizeof gr, "g1r%d", sl);
                    snprintf(gi, sizeof gi, "g1i%d", sl);
                    apply(j, gr, gi);
                } else if (!hi && ((run_g0 >> sl) & 1)) {
                    snprintf(gr, sizeof gr, "g0r%d", sl);
                    snprintf(gi, sizeof gi, "g0i%d", sl);
                    apply(j, gr, gi);
                }
            }
        if (run_all)
            for (int j = 0; j < V; ++j) apply(j, "gar", "gai");
        g.line("    } // diagonal run");
        run_open = false;
    };
    for (int o = 0; o < nops; ++o) {
        const FOp &op = ops[o];
        if (op.kind == OP_CONT) continue;  // rows of the OP_DENSE2 before it
        if (op.kind == OP_DIAG) {
            int creg;
            uint32_t cthr;
            split_ctrl(L, M, op.lctrl, creg, cthr);
            int rslot = -1;
            for (int i = 0; i < M; ++i)
                if (op.lbit >= 0 && L.rb[i] == op.lbit) rslot = i;
            if (creg == 0) {
                if (!run_open) {
                    g.line("    { // diagonal run");
                    for (int sl = 0; sl < M; ++sl)
                        g.line("    %s g1r%d = 1, g1i%d = 0, g0r%d = 1, g0i%d = 0;", R, sl, sl, sl, sl);
                    g.line("    %s gar = 1, gai = 0;", R);
                    run_open = true;
                    run_g1 = run_g0 = 0;
                    run_all = false;
                }
                const bool d0one = op.slot < 0 && op.m[0] == 1.0 && op.m[1] == 0.0;
                const bool d1one = op.slot < 0 && op.m[6] == 1.0 && op.m[7] == 0.0;
                g.line("    { // op %d kind %d (folded)", o, op.kind);
                g.line("    const FOp &cur = op[%d];", o);
                if (op.slot >= 0) {
                    g.line("    const %s *tm = trow + (unsigned long long)cur.slot * 8ull;", R);
                    g.line("    const %s ma = tm[0], mb = tm[1], mg = tm[6], mh = tm[7];", R);
                } else {
                    g.line("    const %s ma = (%s)cur.m[0], mb = (%s)cur.m[1], mg = (%s)cur.m[6], mh = (%s)cur.m[7];", R, R,
                           R, R, R);
                }
                std::string cond = "true";
                if (cthr) {
                    char c[64];
                    snprintf(c, sizeof c, "((tp & %uu) == %uu)", cthr, cthr);
                    cond = c;
                }
                if (op.gctrl) cond += " && ((base & cur.gctrl) == cur.gctrl)";
                g.line("    const bool c = %s;", cond.c_str());
                auto fold = [&](const char *acc, const char *fr, const char *fi) {
                    g.line("    { const %s fr = c ? %s : (%s)1, fi = c ? %s : (%s)0;", R, fr, R, fi, R);
                    g.line("      const %s t = %sr * fr - %si * fi; %si = %sr * fi + %si * fr; %sr = t; }", R, acc, acc, acc,
                           acc, acc, acc);
                };
                if (rslot >= 0) {
                    if (!d1one) {
                        g.line("    { const %s fr = c ? mg : (%s)1, fi = c ? mh : (%s)0;", R, R, R);
                        g.line("      const %s t = g1r%d * fr - g1i%d * fi; g1i%d = g1r%d * fi + g1i%d * fr; g1r%d = t; }", R,
                               rslot, rslot, rslot, rslot, rslot, rslot);
                        run_g1 |= 1u << rslot;
                    }
                    if (!d0one) {
                        g.line("    { const %s fr = c ? ma : (%s)1, fi = c ? mb : (%s)0;", R, R, R);
                        g.line("      const %s t = g0r%d * fr - g0i%d * fi; g0i%d = g0r%d * fi + g0i%d * fr; g0r%d = t; }", R,
                               rslot, rslot, rslot, rslot, rslot, rslot);
                        run_g0 |= 1u << rslot;
                    }
                } else if (!(d0one && d1one)) {
                    if (op.lbit >= 0)
                        g.line("    const bool hi = (tp >> %d) & 1u;", op.lbit);
                    else
                        g.line("    const bool hi = (base & cur.gtbit) != 0ull;");
                    fold("ga", "(hi ? mg : ma)", "(hi ? mh : mb)");
                    run_all = true;
                }
                g.line("    }");
                continue;
            }
        } else if (run_open) {
            close_run();
        }
        if (op.kind == OP_FACTOR) {
            int e = o;
            while (e < nops && ops[e].kind == OP_FACTOR) ++e;
            phase_run(g, ops, o, e, M, c128);
            o = e - 1;
            continue;
        }
        g.line("    { // op %d kind %d", o, op.kind);
        g.line("    const FOp &cur = op[%d];", o);
        if (op.kind == OP_GIVENS) {
            // real rotation with one unit coefficient per row: one
            // multiply-add per real component
            int creg;
            uint32_t cthr;
            split_ctrl(L, M, op.lctrl, creg, cthr);
            int close = 0;
            if (op.gctrl) {
                g.line("    if ((base & cur.gctrl) == cur.gctrl) {");
                ++close;
            }
            if (cthr) {
                g.line("    if ((tp & %uu) == %uu) {", cthr, cthr);
                ++close;
            }
            const char *F = c128 ? "__builtin_fma" : "__builtin_fmaf";
            const int S = op.lbit & 0xff, form = op.lbit >> 8;
            g.line("    const %s t = (%s)cur.m[0], nt = -t;", R, R);
            for (int j = 0; j < V; ++j) {
                if ((j >> S) & 1) continue;
                if ((j & creg) != creg) continue;
                const int jj = j | (1 << S);
                g.line("    { const %s x = v[%d], y = v[%d];", T, j, jj);
                if (form == 0) {
                    g.line("      v[%d].x = %s(nt, y.x, x.x); v[%d].y = %s(nt, y.y, x.y);", j, F, j, F);
                    g.line("      v[%d].x = %s(t, x.x, y.x); v[%d].y = %s(t, x.y, y.y); }", jj, F, jj, F);
                } else {
                    g.line("      v[%d].x = %s(t, x.x, -y.x); v[%d].y = %s(t, x.y, -y.y);", j, F, j, F);
                    g.line("      v[%d].x = %s(t, y.x, x.x); v[%d].y = %s(t, y.y, x.y); }", jj, F, jj, F);
                }
            }
            for (int c = 0; c < close; ++c) g.line("    }");
            g.line("    }");
            continue;
        }
        if (op.kind == OP_DENSE2 && mfma) {
            // 4x4 on register slots lo, hi as two MFMA chains per group of
            // four amplitudes (output rows 0-1, then 2-3), eight steps each
            // over the group's real and imaginary parts (every entry used)
            const int lo = op.lbit & 0xff, hi = op.lbit >> 8;
            for (int h = 0; h < 2; ++h) {
                g.line("    const int rr%d = %d + (ri >> 1); const bool im%d = ri & 1;", h, 2 * h, h);
                for (int c = 0; c < 4; ++c) {
                    g.line("    const float er%d%d = (float)op[%d + rr%d].m[%d], ei%d%d = (float)op[%d + rr%d].m[%d];", h, c,
                           o, h, 2 * c, h, c, o, h, 2 * c + 1);
                    g.line("    const float ar%d%d = im%d ? ei%d%d : er%d%d, ai%d%d = im%d ? er%d%d : -ei%d%d;", h, c, h, h,
                           c, h, c, h, c, h, h, c, h, c);
                }
            }
            std::vector<std::array<int, 4>> grp;
            for (int j = 0; j < V; ++j) {
                if (((j >> lo) & 1) || ((j >> hi) & 1)) continue;
                grp.push_back({j, j | (1 << lo), j | (1 << hi), j | (1 << lo) | (1 << hi)});
            }
            for (size_t q = 0; q < grp.size(); ++q)
                g.line("    v4f d%zu_0 = {0.f, 0.f, 0.f, 0.f}, d%zu_1 = {0.f, 0.f, 0.f, 0.f};", q, q);
            for (int h = 0; h < 2; ++h)
                for (int c = 0; c < 4; ++c) {
                    // skip a column both rows of the chain have as exact zeros
                    const bool z = ((op.lctrl >> (4 * (2 * h) + c)) & 1) && ((op.lctrl >> (4 * (2 * h + 1) + c)) & 1);
                    if (z) continue;
                    for (size_t q = 0; q < grp.size(); ++q) {
                        g.line("    d%zu_%d = __builtin_amdgcn_mfma_f32_4x4x1f32(ar%d%d, v[%d].x, d%zu_%d, 0, 0, 0);", q, h, h,
                               c, grp[q][size_t(c)], q, h);
                        g.line("    d%zu_%d = __builtin_amdgcn_mfma_f32_4x4x1f32(ai%d%d, v[%d].y, d%zu_%d, 0, 0, 0);", q, h, h,
                               c, grp[q][size_t(c)], q, h);
                    }
                }
            for (size_t q = 0; q < grp.size(); ++q) {
                g.line("    v[%d] = c64{d%zu_0[0], d%zu_0[1]}; v[%d] = c64{d%zu_0[2], d%zu_0[3]};", grp[q][0], q, q, grp[q][1],
                       q, q);
                g.line("    v[%d] = c64{d%zu_1[0], d%zu_1[1]}; v[%d] = c64{d%zu_1[2], d%zu_1[3]};", grp[q][2], q, q, grp[q][3],
                       q, q);
            }
            g.line("    }");
            continue;
        }
        if (op.kind == OP_DENSE2) {
            // 4x4 on register slots lo, hi: block index (bit hi) << 1 | (bit lo)
            const int lo = op.lbit & 0xff, hi = op.lbit >> 8;
            for (int r = 0; r < 4; ++r)
                for (int c = 0; c < 4; ++c)
                    if (!((op.lctrl >> (4 * r + c)) & 1))
                        g.line("    const %s m%d%dr = (%s)op[%d].m[%d], m%d%di = (%s)op[%d].m[%d];", R, r, c, R, o + r,
                               2 * c, r, c, R, o + r, 2 * c + 1);
            for (int j = 0; j < V; ++j) {
                if (((j >> lo) & 1) || ((j >> hi) & 1)) continue;
                const int idx[4] = {j, j | (1 << lo), j | (1 << hi), j | (1 << lo) | (1 << hi)};
                g.line("    { const %s x0 = v[%d], x1 = v[%d], x2 = v[%d], x3 = v[%d];", T, idx[0], idx[1], idx[2], idx[3]);
                for (int r = 0; r < 4; ++r) {
                    std::string re = "", im = "";
                    for (int c = 0; c < 4; ++c) {
                        if ((op.lctrl >> (4 * r + c)) & 1) continue;
                        char t1[96], t2[96];
                        snprintf(t1, sizeof t1, "%sm%d%dr * x%d.x - m%d%di * x%d.y", re.empty() ? "" : " + ", r, c, c, r, c,
                                 c);
                        snprintf(t2, sizeof t2, "%sm%d%dr * x%d.y + m%d%di * x%d.x", im.empty() ? "" : " + ", r, c, c, r, c,
                                 c);
                        re += t1;
                        im += t2;
                    }
                    if (re.empty()) {
                        re = "0";
                        im = "0";
                    }
                    g.line("      v[%d].x = %s;", idx[r], re.c_str());
                    g.line("      v[%d].y = %s;", idx[r], im.c_str());
                }
                g.line("    }");
            }
            g.line("    }");
            continue;
        }
        if (op.kind == OP_REMAP) {
            // The swizzle is linear over the bits and the thread and
            // register parts of an index are disjoint, so the LDS byte
            // offset of register j is swz(tp) * size ^ swz(reg part) * size:
            // one XOR with a constant per register.  The lane part is
            // opaque to keep the compiler from folding the shift back
            // into every register's address.
            if (lds_live) g.line("    lds_barrier();");
            g.line("    { unsigned sw = %s * %du; asm(\"\" : \"+v\"(sw));", swz("tp").c_str(), int(sizeof(double)) * (c128 ? 2 : 1));
            for (int j = 0; j < V; ++j)
                g.line("      *(%s *)((char *)lds + (sw ^ %uu)) = v[%d];", T, swz_const(reg_off(L, M, j)) * (c128 ? 16u : 8u), j);
            g.line("    }");
            g.line("    lds_barrier();");
            for (int i = 0; i < M; ++i) L.rb[i] = int((op.lctrl >> (4 * i)) & 15u);
            g.line("    tp = %s;", deposit_expr(K, M, L).c_str());
            g.line("    { unsigned sw = %s * %du; asm(\"\" : \"+v\"(sw));", swz("tp").c_str(), int(sizeof(double)) * (c128 ? 2 : 1));
            for (int j = 0; j < V; ++j)
                g.line("      v[%d] = *(const %s *)((const char *)lds + (sw ^ %uu));", j, T,
                       swz_const(reg_off(L, M, j)) * (c128 ? 16u : 8u));
            g.line("    }");
            lds_live = true;
            g.line("    }");
            continue;
        }
        int creg;
        uint32_t cthr;
        split_ctrl(L, M, op.lctrl, creg, cthr);
        int close = 0;
        if (op.gctrl) {
            g.line("    if ((base & cur.gctrl) == cur.gctrl) {");
            ++close;
        }
        if (op.kind != OP_PERM && op.slot >= 0) {
            // per-register matrix: row cur.slot of this register's table
            g.line("    const %s *tm = trow + (unsigned long long)cur.slot * 8ull;", R);
            g.line("    const %s ma = tm[0], mb = tm[1], mc = tm[2], md = tm[3];", R);
            g.line("    const %s me = tm[4], mf = tm[5], mg = tm[6], mh = tm[7];", R);
        } else if (op.kind != OP_PERM) {
            g.line("    const %s ma = (%s)cur.m[0], mb = (%s)cur.m[1], mc = (%s)cur.m[2], md = (%s)cur.m[3];", R, R, R, R,
                   R);
            g.line("    const %s me = (%s)cur.m[4], mf = (%s)cur.m[5], mg = (%s)cur.m[6], mh = (%s)cur.m[7];", R, R, R, R,
                   R);
        }
        if (cthr) {
            g.line("    if ((tp & %uu) == %uu) {", cthr, cthr);
            ++close;
        }
        if (op.kind == OP_DENSE && mfma && !cthr) {
            // v_mfma_f32_4x4x1_16b: 16 blocks D(4x4) += A(4x1) B(1x4), block
            // b = lanes 4b..4b+3; lane 4b+j holds B[j] and column j of D,
            // lane 4b+i holds A[i].  With B = one real component x_k of the
            // lane's own pair (x = v[j], y = v[jj]; k = x.re, x.im, y.re,
            // y.im) and A = entry (ri, k) of the pair's real 4x4 matrix, four
            // steps leave the lane's D = (x'.re, x'.im, y'.re, y'.im).
            // Lanes never mix their amplitudes, so no exchange is needed and
            // the matrix-core work equals the 16 multiply-adds per pair.
            const int S = op.lbit;
            g.line("    const bool top = ri < 2, odd = ri & 1;");
            g.line("    const float p0 = top ? ma : me, p1 = top ? mb : mf, p2 = top ? mc : mg, p3 = top ? md : mh;");
            g.line("    const float A0 = odd ? p1 : p0, A1 = odd ? p0 : -p1, A2 = odd ? p3 : p2, A3 = odd ? p2 : -p3;");
            std::vector<std::pair<int, int>> pr;
            for (int j = 0; j < V; ++j) {
                if ((j >> S) & 1) continue;
                if ((j & creg) != creg) continue;
                pr.push_back({j, j | (1 << S)});
            }
            for (size_t q = 0; q < pr.size(); ++q) g.line("    v4f d%zu = {0.f, 0.f, 0.f, 0.f};", q);
            const char *Av[4] = {"A0", "A1", "A2", "A3"};
            for (int k = 0; k < 4; ++k)
                for (size_t q = 0; q < pr.size(); ++q)
                    g.line("    d%zu = __builtin_amdgcn_mfma_f32_4x4x1f32(%s, v[%d].%s, d%zu, 0, 0, 0);", q, Av[k],
                           k < 2 ? pr[q].first : pr[q].second, (k & 1) ? "y" : "x", q);
            for (size_t q = 0; q < pr.size(); ++q)
                g.line("    v[%d] = c64{d%zu[0], d%zu[1]}; v[%d] = c64{d%zu[2], d%zu[3]};", pr[q].first, q, q, pr[q].second,
                       q, q);
        } else if (op.kind == OP_DENSE || op.kind == OP_PERM) {
            const int S = op.lbit;
            for (int j = 0; j < V; ++j) {
                if ((j >> S) & 1) continue;
                if ((j & creg) != creg) continue;
                const int jj = j | (1 << S);
                if (op.kind == OP_PERM) {
                    g.line("    { const %s x = v[%d]; v[%d] = v[%d]; v[%d] = x; }", T, j, j, jj, jj);
                } else {
                    g.line("    { const %s x = v[%d], y = v[%d];", T, j, jj);
                    g.line("      v[%d].x = ma * x.x - mb * x.y + mc * y.x - md * y.y;", j);
                    g.line("      v[%d].y = ma * x.y + mb * x.x + mc * y.y + md * y.x;", j);
                    g.line("      v[%d].x = me * x.x - mf * x.y + mg * y.x - mh * y.y;", jj);
                    g.line("      v[%d].y = me * x.y + mf * x.x + mg * y.y + mh * y.x; }", jj);
                }
            }
        } else {  // OP_DIAG
            // entries known to be 1 are skipped; a table matrix is not known here
            const bool d0one = op.slot < 0 && op.m[0] == 1.0 && op.m[1] == 0.0;
            const bool d1one = op.slot < 0 && op.m[6] == 1.0 && op.m[7] == 0.0;
            const int lb = op.lbit;
            int rslot = -1;
            for (int i = 0; i < M; ++i)
                if (lb >= 0 && L.rb[i] == lb) rslot = i;
            auto scale = [&](int j, const char *fr, const char *fi) {
                g.line("    { const %s x = v[%d]; v[%d].x = %s * x.x - %s * x.y; v[%d].y = %s * x.y + %s * x.x; }", T, j,
                       j, fr, fi, j, fr, fi);
            };
            if (rslot >= 0) {
                for (int j = 0; j < V; ++j) {
                    if ((j & creg) != creg) continue;
                    const bool hi = (j >> rslot) & 1;
                    if (hi ? d1one : d0one) continue;
                    scale(j, hi ? "mg" : "ma", hi ? "mh" : "mb");
                }
            } else if (!(d0one && d1one)) {
                if (lb >= 0) {
                    g.line("    const bool hi = (tp >> %d) & 1u;", lb);
                } else {
                    g.line("    const bool hi = (base & cur.gtbit) != 0ull;");
                }
                g.line("    const %s fr = hi ? mg : ma, fi = hi ? mh : mb;", R);
                if (lb < 0) {
                    g.line("    if (!(fr == (%s)1 && fi == (%s)0)) {", R, R);
                    ++close;
                }
                for (int j = 0; j < V; ++j) {
                    if ((j & creg) != creg) continue;
                    scale(j, "fr", "fi");
                }
            }
        }
        for (int c = 0; c < close; ++c) g.line("    }");
        g.line("    }");
    }
    close_run();
    // the planner ends every pass in the canonical layout
    if (cbits) {
        for (int j = 0; j < V; ++j)
            g.line("    __builtin_nontemporal_store(v[%d], a + (gth | %lluull));", j, gj[size_t(j)]);
    } else {
        run_time_index("__builtin_nontemporal_store(v[j], a + gi);");
    }
    g.line("}");
    return g.s;
}

// Everything the generator reads from a pass, packed into a string: two
// passes with the same signature get the same kernel source.
std::string signature(int dtype, int M, const FPass &P, const FOp *ops, bool mfma_on, int waves) {
    std::string k;
    k.reserve(16 + size_t(P.nops) * 16);
    auto put = [&](uint32_t x) { k.append(reinterpret_cast<const char *>(&x), sizeof x); };
    put(uint32_t(dtype));
    put(uint32_t(dtype == SV_C64 && mfma_on));
    put(uint32_t(waves));
    put(uint32_t(M));
    put(uint32_t(P.k));
    put(uint32_t(P.nops));
    bool table = false;
    for (int o = 0; o < P.nops; ++o) {
        const FOp &x = ops[P.first + o];
        table |= (x.kind == OP_DENSE || x.kind == OP_DIAG) && x.slot >= 0;  // per-trajectory matrix
    }
    if (!table || svi_config().batch_const_bits) {  // plain passes compile their tile bits in as constants
        put(uint32_t(P.nlow));
        for (int i = 0; i < P.k; ++i) put(uint32_t(uint8_t(P.bits[i])));
    }
    for (int o = 0; o < P.nops; ++o) {
        const FOp &op = ops[P.first + o];
        const bool d0one = op.kind == OP_DIAG && op.slot < 0 && op.m[0] == 1.0 && op.m[1] == 0.0;
        const bool d1one = op.kind == OP_DIAG && op.slot < 0 && op.m[6] == 1.0 && op.m[7] == 0.0;
        put(uint32_t(op.kind));
        put(uint32_t(op.lbit));
        put(op.lctrl);
        put(uint32_t(op.slot >= 0) | uint32_t(op.gctrl != 0) << 1 | uint32_t(d0one) << 2 | uint32_t(d1one) << 3);
    }
    return k;
}

struct JitCache {
    std::mutex mu;
    std::unordered_map<std::string, std::vector<char>> code;  // signature -> code object
    std::unordered_map<std::string, hipFunction_t> fn;        // device + signature -> kernel
    std::string last_error;
};

JitCache &cache() {
    static JitCache *c = new JitCache();  // kept to process exit (modules stay loaded)
    return *c;
}

bool compile(const std::string &src, std::vector<char> &out, std::string &err) {
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "sv_pass.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) {
        err = "hiprtcCreateProgram failed";
        return false;
    }
    // packed FP32 instructions stay disabled, as for the library's own kernels
    const char *opts[] = {"--offload-arch=gfx950", "-O3", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult rc = hiprtcCompileProgram(prog, int(sizeof(opts) / sizeof(opts[0])), opts);
    bool ok = rc == HIPRTC_SUCCESS;
    if (!ok) {
        size_t n = 0;
        hiprtcGetProgramLogSize(prog, &n);
        std::string log(n, '\0');
        if (n) hiprtcGetProgramLog(prog, &log[0]);
        err = std::string("hiprtc: ") + hiprtcGetErrorString(rc) + ": " + log.substr(0, 400);
    } else {
        size_t n = 0;
        ok = hiprtcGetCodeSize(prog, &n) == HIPRTC_SUCCESS && n > 0;
        if (ok) {
            out.resize(n);
            ok = hiprtcGetCode(prog, out.data()) == HIPRTC_SUCCESS;
        }
        if (!ok) err = "hiprtcGetCode failed";
    }
    hiprtcDestroyProgram(&prog);
    return ok;
}

}  // namespace

int svi_jit_kmax(int dtype) { return dtype == SV_C128 ? 12 : 13; }

// Kernels of every pass of prog on the current device (compiled on first use,
// in parallel).
namespace {
bool is_generic(const FusedProgram &prog, size_t p) { return p < prog.generic.size() && prog.generic[p]; }
}  // namespace

int svi_jit_prepare(int device, int dtype, const FusedProgram &prog, std::vector<hipFunction_t> &fns) {
    JitCache &C = cache();
    // modules load into the current device's context; a wrapped register
    // does not record its device
    if (device < 0) {
        const hipError_t e = hipGetDevice(&device);
        if (e != hipSuccess) return svi_fail("sv_run: current device", e);
    }
    const size_t np = prog.passes.size();
    std::vector<std::string> sig(np);
    for (size_t p = 0; p < np; ++p)
        sig[p] = signature(dtype, std::min(prog.m, int(prog.passes[p].k)), prog.passes[p], prog.ops.data(), svi_prog_mfma(prog),
                           svi_prog_waves(prog));
    // passes whose kernel has not been compiled yet, one per signature
    std::vector<size_t> todo;
    {
        std::lock_guard<std::mutex> lk(C.mu);
        std::unordered_set<std::string> seen;
        for (size_t p = 0; p < np; ++p)
            if (!is_generic(prog, p) && !C.code.count(sig[p]) && seen.insert(sig[p]).second) todo.push_back(p);
    }
    if (!todo.empty()) {
        std::vector<std::vector<char>> objs(todo.size());
        std::vector<std::string> errs(todo.size());
        std::vector<char> oks(todo.size(), 0);
        const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
        const size_t nthr = std::min<size_t>(todo.size(), std::min(16u, hw));
        std::vector<std::thread> th;
        for (size_t w = 0; w < nthr; ++w)
            th.emplace_back([&, w] {
                for (size_t i = w; i < todo.size(); i += nthr) {
                    const FPass &P = prog.passes[todo[i]];
                    const std::string src =
                        generate(dtype, P.k, std::min(prog.m, P.k), P, prog.ops.data() + P.first, P.nops, svi_prog_mfma(prog),
                        svi_prog_waves(prog));
                    oks[i] = compile(src, objs[i], errs[i]);
                }
            });
        for (auto &x : th) x.join();
        std::lock_guard<std::mutex> lk(C.mu);
        for (size_t i = 0; i < todo.size(); ++i) {
            if (!oks[i]) {
                C.last_error = errs[i];
                return svi_fail_text(("pass compilation failed: " + errs[i]).c_str(), SV_EDEVICE);
            }
            C.code[sig[todo[i]]] = std::move(objs[i]);
        }
    }
    fns.assign(np, nullptr);
    std::lock_guard<std::mutex> lk(C.mu);
    const std::string dev = std::to_string(device) + ":";
    for (size_t p = 0; p < np; ++p) {
        if (is_generic(prog, p)) continue;  // stays nullptr: the caller launches the generic kernel
        const std::string key = dev + sig[p];
        auto it = C.fn.find(key);
        if (it == C.fn.end()) {
            hipModule_t mod;
            hipFunction_t f;
            hipError_t e = hipModuleLoadData(&mod, C.code[sig[p]].data());
            if (e == hipSuccess) e = hipModuleGetFunction(&f, mod, "sv_pass");
            if (e != hipSuccess) return svi_fail("loading a compiled pass", e);
            it = C.fn.emplace(key, f).first;
        }
        fns[p] = it->second;
    }
    return SV_OK;
}

hipError_t svi_jit_launch(hipFunction_t f, const FusedLaunch &L, int K, int M, const FPass *dpass, const FOp *dops) {
    int tile_bits = L.n - K;
    if (tile_bits < 0 || tile_bits > 31 || L.nregs == 0) return hipErrorInvalidValue;
    const uint64_t grid = L.nregs << tile_bits;
    if ((L.nregs >> (31 - tile_bits)) != 0 || grid > 0x7fffffffull) return hipErrorInvalidValue;
    void *a = L.state;
    const void *p = dpass;
    const void *o = dops;
    const void *tb = L.table;
    unsigned nslots = L.nslots;
    int n = L.n;
    void *args[] = {&a, &p, &o, &tb, &nslots, &tile_bits, &n};
    return hipModuleLaunchKernel(f, unsigned(grid), 1, 1, 1u << (K - M), 1, 1, 0, L.stream, args, nullptr);
}

// Source of the kernel of one pass (host only; for inspection and tests).
std::string svi_jit_pass_source(int dtype, const FusedProgram &prog, size_t pass) {
    const FPass &P = prog.passes[pass];
    return generate(dtype, P.k, std::min(prog.m, P.k), P, prog.ops.data() + P.first, P.nops, svi_prog_mfma(prog),
                        svi_prog_waves(prog));
}

extern "C" int sv_jit_source(int n, int dtype, const sv_gate *gates, int64_t ng, int64_t pass, char *buf,
                             int64_t cap, int64_t *len) {
    if (n < 1 || n > SV_MAX_QUBITS || (dtype != SV_C64 && dtype != SV_C128) || ng < 0 || (ng > 0 && !gates) ||
        !len || pass < 0)
        return SV_EINVAL;
    std::vector<PreparedGate> prep;
    int rc = svi_prepare(n, gates, ng, prep, nullptr);
    if (rc != SV_OK) return rc;
    FusedProgram prog;
    rc = svi_fused_compile(n, dtype, prep.data(), ng, prog);
    if (rc != SV_OK) return rc;
    svi_jit_transform(prog);
    if (pass >= int64_t(prog.passes.size())) return SV_EINVAL;
    const FPass &P = prog.passes[size_t(pass)];
    const std::string s = generate(dtype, P.k, std::min(prog.m, P.k), P, prog.ops.data() + P.first, P.nops, svi_prog_mfma(prog),
                        svi_prog_waves(prog));
    *len = int64_t(s.size());
    if (buf && cap > 0) {
        const size_t m = std::min<size_t>(s.size(), size_t(cap - 1));
        std::memcpy(buf, s.data(), m);
        buf[m] = '\0';
    }
    return SV_OK;
}

// ------------------------------------------------------------ pair fusion
//
// Inside a pass, between two layout changes, every op acts on register
// slots and thread bits of a fixed layout.  Ops whose target and in-tile
// controls all sit on at most two register slots, with no out-of-tile
// control and no per-register matrix, can be multiplied into one 2x2 or
// 4x4 matrix (in FP64, rounded once by the kernel).  A dense 4x4 costs 16
// multiply-adds per amplitude against 8 for each dense 2x2 it replaces, so
// a run of two SU(2) layers around a CNOT halves the arithmetic; runs are
// only fused when the composed matrix (by its nonzero entries) is cheaper
// than its members.  Ops on other slots commute with a run and may sit
// between its members; an op that touches a run's slots without joining it
// closes the run, which is then emitted at that point.

namespace {

using cplx = std::complex<double>;

struct Group {
    int lo = -1, hi = -1;       // register slots (hi = -1: one slot)
    std::vector<FOp> members;   // in program order
};

// Slots of the register bits in a local mask; false if any bit is a thread bit.
bool reg_slots_of(const int *slot_of, uint32_t mask, uint32_t &slots) {
    slots = 0;
    bool all = true;
    for (uint32_t m = mask; m; m &= m - 1) {
        const int b = __builtin_ctz(m);
        if (slot_of[b] < 0)
            all = false;
        else
            slots |= 1u << slot_of[b];
    }
    return all;
}

double op_cost(const FOp &op) {
    if (op.kind == OP_DENSE) return 8.0;
    if (op.kind == OP_DIAG) return 4.0;
    return 0.0;  // exchanges are register renamings
}

// Matrix of op on the group's slots (index bit 0 = lo, bit 1 = hi); D = 2 or 4.
void op_matrix(const FOp &op, const int *slot_of, int lo, int hi, int D, std::vector<cplx> &G) {
    G.assign(size_t(D) * D, cplx(0, 0));
    auto pos_of_slot = [&](int s) { return s == lo ? 0 : 1; };
    int p;  // target position
    if (op.kind == OP_DIAG)
        p = pos_of_slot(slot_of[op.lbit]);
    else
        p = pos_of_slot(op.lbit);
    int cm = 0;
    for (uint32_t m = op.lctrl; m; m &= m - 1) cm |= 1 << pos_of_slot(slot_of[__builtin_ctz(m)]);
    (void)hi;
    const cplx u[2][2] = {{cplx(op.m[0], op.m[1]), cplx(op.m[2], op.m[3])},
                          {cplx(op.m[4], op.m[5]), cplx(op.m[6], op.m[7])}};
    for (int c = 0; c < D; ++c) {
        if ((c & cm) != cm) {
            G[size_t(c) * D + c] = 1.0;
            continue;
        }
        const int bit = (c >> p) & 1;
        if (op.kind == OP_DIAG) {
            G[size_t(c) * D + c] = bit ? u[1][1] : u[0][0];
        } else if (op.kind == OP_PERM) {
            G[size_t(c ^ (1 << p)) * D + c] = 1.0;
        } else {
            const int c0 = c & ~(1 << p), c1 = c | (1 << p);
            G[size_t(c0) * D + c] = u[0][bit];
            G[size_t(c1) * D + c] = u[1][bit];
        }
    }
}

void emit_group(const Group &g, const int *slot_of, const int *rb, std::vector<FOp> &out) {
    if (g.members.size() < 2) {
        for (const FOp &o : g.members) out.push_back(o);
        return;
    }
    const int D = g.hi < 0 ? 2 : 4;
    std::vector<cplx> M(size_t(D) * D, cplx(0, 0)), G, T(size_t(D) * D);
    for (int i = 0; i < D; ++i) M[size_t(i) * D + i] = 1.0;
    double cost = 0.0;
    for (const FOp &o : g.members) {
        cost += op_cost(o);
        op_matrix(o, slot_of, g.lo, g.hi, D, G);
        for (int r = 0; r < D; ++r)
            for (int c = 0; c < D; ++c) {
                cplx acc = 0.0;
                for (int k = 0; k < D; ++k) acc += G[size_t(r) * D + k] * M[size_t(k) * D + c];
                T[size_t(r) * D + c] = acc;
            }
        M.swap(T);
    }
    int nnz = 0;
    for (const cplx &x : M) nnz += x != cplx(0, 0);
    const bool diag = D == 2 && M[1] == cplx(0, 0) && M[2] == cplx(0, 0);
    // multiply-adds per amplitude: nnz complex products spread over D rows
    const double fused_cost = diag ? 4.0 : 4.0 * nnz / D;
    if (!(fused_cost < cost)) {
        for (const FOp &o : g.members) out.push_back(o);
        return;
    }
    FOp h;
    std::memset(&h, 0, sizeof h);
    h.slot = -1;
    if (D == 2) {
        h.kind = diag ? OP_DIAG : OP_DENSE;
        h.lbit = diag ? rb[g.lo] : g.lo;
        for (int i = 0; i < 4; ++i) {
            h.m[2 * i] = M[size_t(i)].real();
            h.m[2 * i + 1] = M[size_t(i)].imag();
        }
        out.push_back(h);
        return;
    }
    h.kind = OP_DENSE2;
    h.lbit = g.lo | (g.hi << 8);
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c)
            if (M[size_t(r) * 4 + c] == cplx(0, 0)) h.lctrl |= 1u << (4 * r + c);
    for (int r = 0; r < 4; ++r) {
        FOp rec = h;
        if (r) {
            std::memset(&rec, 0, sizeof rec);
            rec.kind = OP_CONT;
            rec.slot = -1;
        }
        for (int c = 0; c < 4; ++c) {
            rec.m[2 * c] = M[size_t(r) * 4 + c].real();
            rec.m[2 * c + 1] = M[size_t(r) * 4 + c].imag();
        }
        out.push_back(rec);
    }
}

}  // namespace

void svi_jit_fuse_pairs(FusedProgram &prog, bool one_slot, const std::vector<char> *only) {
    std::vector<FOp> out;
    out.reserve(prog.ops.size());
    for (size_t pi = 0; pi < prog.passes.size(); ++pi) {
        FPass &P = prog.passes[pi];
        if ((pi < prog.generic.size() && prog.generic[pi]) || (only && !(*only)[pi])) {
            // left to the generic kernel, which knows no composed ops
            const size_t first = out.size();
            out.insert(out.end(), prog.ops.begin() + P.first, prog.ops.begin() + P.first + P.nops);
            P.first = int32_t(first);
            continue;
        }
        const int K = P.k, M = std::min(prog.m, K);
        int rb[4];
        int slot_of[32];
        auto set_layout = [&](const int *nrb) {
            for (int b = 0; b < 32; ++b) slot_of[b] = -1;
            for (int i = 0; i < M; ++i) {
                rb[i] = nrb[i];
                slot_of[rb[i]] = i;
            }
        };
        int canon[4];
        for (int i = 0; i < M; ++i) canon[i] = K - M + i;
        set_layout(canon);
        const size_t first = out.size();
        std::vector<Group> open;
        auto close_touching = [&](uint32_t slots) {
            for (size_t i = 0; i < open.size();) {
                const uint32_t gs = (1u << open[i].lo) | (open[i].hi >= 0 ? 1u << open[i].hi : 0u);
                if (gs & slots) {
                    emit_group(open[i], slot_of, rb, out);
                    open.erase(open.begin() + long(i));
                } else {
                    ++i;
                }
            }
        };
        for (int o = 0; o < P.nops; ++o) {
            const FOp &op = prog.ops[size_t(P.first + o)];
            if (op.kind == OP_REMAP) {
                close_touching(0xF);
                out.push_back(op);
                int nrb[4];
                for (int i = 0; i < M; ++i) nrb[i] = int((op.lctrl >> (4 * i)) & 15u);
                set_layout(nrb);
                continue;
            }
            // register slots the op involves, and whether it may join a run
            uint32_t cslots = 0;
            const bool ctrl_in_regs = reg_slots_of(slot_of, op.lctrl, cslots);
            int tslot = -1;
            if (op.kind == OP_DIAG)
                tslot = op.lbit >= 0 ? slot_of[op.lbit] : -1;
            else
                tslot = op.lbit;
            const uint32_t touched = cslots | (tslot >= 0 ? 1u << tslot : 0u);
            const bool joinable = tslot >= 0 && ctrl_in_regs && op.gctrl == 0 && op.slot < 0 &&
                                  !(op.kind == OP_DIAG && op.gtbit != 0) &&
                                  __builtin_popcount(touched) <= (one_slot ? 1 : 2);
            if (!joinable) {
                close_touching(touched);
                out.push_back(op);
                continue;
            }
            // the runs holding the op's slots
            std::vector<size_t> hit;
            for (size_t i = 0; i < open.size(); ++i) {
                const uint32_t gs = (1u << open[i].lo) | (open[i].hi >= 0 ? 1u << open[i].hi : 0u);
                if (gs & touched) hit.push_back(i);
            }
            const bool pair = __builtin_popcount(touched) == 2;
            if (!pair) {
                if (hit.empty()) {
                    Group g;
                    g.lo = tslot;
                    g.members.push_back(op);
                    open.push_back(g);
                } else {
                    open[hit[0]].members.push_back(op);
                }
                continue;
            }
            const int a = __builtin_ctz(touched), b = 31 - __builtin_clz(touched);
            // join an open run on exactly these slots, or merge one-slot runs on them
            bool ok = true;
            for (size_t i : hit)
                if (open[i].hi >= 0 && !(open[i].lo == a && open[i].hi == b)) ok = false;
            if (!ok) {
                close_touching(touched);
                hit.clear();
            }
            Group g;
            g.lo = a;
            g.hi = b;
            // members of the merged runs keep their program order per slot;
            // runs on different slots commute, so concatenation is valid
            for (size_t i : hit)
                for (const FOp &m : open[i].members) g.members.push_back(m);
            for (size_t k = hit.size(); k-- > 0;) open.erase(open.begin() + long(hit[k]));
            g.members.push_back(op);
            open.push_back(g);
        }
        close_touching(0xF);
        P.first = int32_t(first);
        P.nops = int32_t(out.size() - first);
    }
    prog.ops.swap(out);
}
