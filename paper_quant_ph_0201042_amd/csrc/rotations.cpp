// Unitary one-qubit ops of a specialised pass as phase, real rotation,
// phase; and the phases of a pass merged into a few runs.
//
// A fused pass of complex128 is bound by FP64 vector issue, not by HBM: a
// dense 2x2 costs 16 multiply-adds per amplitude pair (sec. 2.2.1's
// evolution step written out in real arithmetic).  Every unitary 2x2 U
// factors as
//     U = e^{i theta/2} diag(e^{iu}, e^{-iu}) R(x) diag(e^{iv}, e^{-iv}),
// R(x) = [[cos x, -sin x], [sin x, cos x]] (theta = arg det U, the Euler
// angles of the SU(2) part).  R(x) equals cos x [[1, -t], [t, 1]] with
// t = tan x when |cos x| >= |sin x|, else sin x [[t, -1], [1, t]] with
// t = cot x (|t| <= 1 either way, so no coefficient grows): an OP_GIVENS op
// is one multiply-add per real component, 4 per pair instead of 16, and
// its scale goes into the phase after it.  The phases are diagonal, so they
// commute with each other and with every op that acts diagonally on their
// bits; each may sit anywhere between the last and the next op acting
// non-diagonally on one of its bits (its window).  Choosing the fewest
// points that stab every window (greedy by window end, which is optimal for
// intervals) gives the runs; a run is emitted as OP_FACTOR terms that the
// kernel multiplies into one phase per register.
//
// Only passes whose matrices are all known on the host (no per-trajectory
// tables) are rewritten; a matrix that is not unitary to 1e-12 (a
// projector, say) keeps its dense op.
#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <tuple>
#include <vector>

#include "fused.h"

namespace {

using cplx = std::complex<double>;

// A diagonal on one target bit, applied where the controls hold.
struct Phase {
    int tb = -1;      // local target bit, or -1: the target is outside the tile (gt)
    uint64_t gt = 0;  // global target bit when tb < 0
    uint32_t lc = 0;  // controls inside the tile, as local bits
    uint64_t gc = 0;  // controls outside the tile, as global bits
    cplx d0, d1;      // factors for target value 0 and 1
};

struct Item {
    bool phase = false;
    Phase p;
    std::vector<FOp> ops;  // a non-phase item: its op (and OP_CONT rows)
    uint32_t nset = 0;     // local bits it acts on non-diagonally
    bool perm = false;     // an exact NOT on bit nset under controls pl, pgc
    uint32_t pl = 0;
    uint64_t pgc = 0;
};

uint32_t qbits(const std::vector<Phase> &c) {
    uint32_t q = 0;
    for (const Phase &p : c) q |= (p.tb >= 0 ? 1u << p.tb : 0u) | p.lc;
    return q;
}

// Moves the phase components c across item x (either direction): true if
// they commute with it, or if x is a controlled NOT on the target bit of
// some components and a control of none.  A phase (d0, d1) on bit b moved
// across a NOT on b under controls C becomes itself times the phase
// (d1/d0, d0/d1) on b under its own controls and C (the NOT exchanges d0
// and d1 where C holds), so crossing adds that component.
bool cross(std::vector<Phase> &c, const Item &x) {
    if (!(x.nset & qbits(c))) return true;
    if (!x.perm) return false;
    const int p = __builtin_ctz(x.nset);
    for (const Phase &y : c)
        if ((y.lc >> p) & 1) return false;
    const size_t nc = c.size();
    if (nc > 16) return false;
    for (size_t i = 0; i < nc; ++i)
        if (c[i].tb == p) {
            Phase z = c[i];
            z.lc |= x.pl;
            z.gc |= x.pgc;
            z.d0 = c[i].d1 / c[i].d0;
            z.d1 = c[i].d0 / c[i].d1;
            c.push_back(z);
        }
    return true;
}

// U (FOp row-major order) = diag(l0, l1) G diag(r0, r1) with G = [[1, -t], [t, 1]]
// (form 0) or [[t, -1], [1, t]] (form 1).  False if U is not unitary to
// 1e-12 or the factors do not reproduce it to 1e-14.
bool split(const double *m, cplx &r0, cplx &r1, double &t, int &form, cplx &l0, cplx &l1) {
    const cplx A(m[0], m[1]), B(m[2], m[3]), C(m[4], m[5]), D(m[6], m[7]);
    const double e1 = std::abs(std::norm(A) + std::norm(C) - 1.0);
    const double e2 = std::abs(std::norm(B) + std::norm(D) - 1.0);
    const double e3 = std::abs(std::conj(A) * B + std::conj(C) * D);
    if (!(e1 <= 1e-12 && e2 <= 1e-12 && e3 <= 1e-12)) return false;
    const cplx h = std::polar(1.0, 0.5 * std::arg(A * D - B * C));  // h^2 = det U
    const cplx hc = std::conj(h);
    // V = conj(h) U lies in SU(2): [[al, -conj(be)], [be, conj(al)]]
    const cplx al = 0.5 * (hc * A + std::conj(hc * D));
    const cplx be = 0.5 * (hc * C - std::conj(hc * B));
    double c = std::abs(al), s = std::abs(be);
    const double r = std::hypot(c, s);
    if (!(r > 0.5)) return false;
    c /= r;
    s /= r;
    const double pa = c > 0 ? std::arg(al) : 0.0, pb = s > 0 ? std::arg(be) : 0.0;
    const double u = 0.5 * (pa - pb), v = 0.5 * (pa + pb);
    double scale;
    if (c >= s) {
        form = 0;
        t = s / c;
        scale = c;
    } else {
        form = 1;
        t = c / s;
        scale = s;
    }
    r0 = std::polar(1.0, v);
    r1 = std::polar(1.0, -v);
    l0 = h * std::polar(scale, u);
    l1 = h * std::polar(scale, -u);
    const double G[2][2] = {{form ? t : 1.0, form ? -1.0 : -t}, {form ? 1.0 : t, form ? t : 1.0}};
    const cplx L[2] = {l0, l1}, R[2] = {r0, r1}, U[2][2] = {{A, B}, {C, D}};
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            if (std::abs(L[i] * G[i][j] * R[j] - U[i][j]) > 1e-14) return false;
    return true;
}

struct Term {
    uint32_t mask;  // register slots that must all be 1
    int sel;        // -1: none; 0..15: thread local bit; 64: the global bit gsel
    uint64_t gsel;
    uint32_t ct;  // thread local bits that must be 1
    uint64_t gc;  // global bits that must be 1
    cplx v0, v1;  // factor (v1 where the selector bit is 1)
};

// The terms of a run of phases under the register layout slot_of: merged
// by (slots, selector, conditions), plain factors folded into selector terms
// of the same conditions, exact ones dropped.
std::vector<Term> run_terms(const std::vector<Phase> &run, const int *slot_of) {
    std::vector<Term> terms;
    auto add = [&](uint32_t mask, int sel, uint64_t gsel, uint32_t ct, uint64_t gc, cplx v0, cplx v1) {
        for (Term &x : terms)
            if (x.mask == mask && x.sel == sel && x.gsel == gsel && x.ct == ct && x.gc == gc) {
                x.v0 *= v0;
                x.v1 *= v1;
                return;
            }
        terms.push_back(Term{mask, sel, gsel, ct, gc, v0, v1});
    };
    for (const Phase &p : run) {
        uint32_t cm = 0, ct = 0;
        for (uint32_t m = p.lc; m; m &= m - 1) {
            const int b = __builtin_ctz(m);
            if (slot_of[b] >= 0)
                cm |= 1u << slot_of[b];
            else
                ct |= 1u << b;
        }
        if (p.tb >= 0 && slot_of[p.tb] >= 0) {
            // d0 on every register of the controls, d1/d0 where the target slot is 1 too
            add(cm, -1, 0, ct, p.gc, p.d0, p.d0);
            const cplx q = p.d1 / p.d0;
            add(cm | 1u << slot_of[p.tb], -1, 0, ct, p.gc, q, q);
        } else if (p.tb >= 0) {
            add(cm, p.tb, 0, ct, p.gc, p.d0, p.d1);
        } else {
            add(cm, 64, p.gt, ct, p.gc, p.d0, p.d1);
        }
    }
    for (size_t i = 0; i < terms.size();) {
        Term &x = terms[i];
        bool folded = false;
        if (x.sel < 0)
            for (Term &y : terms)
                if (&y != &x && y.sel >= 0 && y.mask == x.mask && y.ct == x.ct && y.gc == x.gc) {
                    y.v0 *= x.v0;
                    y.v1 *= x.v0;
                    folded = true;
                    break;
                }
        if (folded || (x.v0 == cplx(1, 0) && x.v1 == cplx(1, 0)))
            terms.erase(terms.begin() + long(i));
        else
            ++i;
    }
    return terms;
}

bool all_constant(const std::vector<Term> &terms) {
    for (const Term &x : terms)
        if (x.sel >= 0 || x.ct || x.gc) return false;
    return true;
}

// Complex multiplies per thread that the kernel spends on a run (V
// registers): a table run multiplies each register once; otherwise each
// term is multiplied into its accumulator (selector and conditions cost
// about as much again), the per-slot products are spread over the registers
// by a tree over the slots involved, multi-slot terms hit their registers,
// and each register takes its factor.
double run_cost(const std::vector<Term> &terms, int V) {
    if (terms.empty()) return 0.0;
    if (all_constant(terms)) return double(V);
    uint32_t B = 0;
    double c = 0.0;
    for (const Term &x : terms) {
        B |= x.mask;
        c += 1.0 + ((x.sel >= 0 || x.ct || x.gc) ? 1.0 : 0.0);
        if (__builtin_popcount(x.mask) >= 2) c += double(V >> __builtin_popcount(x.mask));
    }
    return c + double((1 << __builtin_popcount(B)) - 1) + double(V);
}

// The OP_FACTOR ops of a run (terms from run_terms) with M register slots.
void emit_run(const std::vector<Term> &terms, int M, std::vector<FOp> &out) {
    if (terms.empty()) return;
    if (all_constant(terms)) {
        // every factor is known here: one table entry per register, four
        // entries per op (selector code 254, lbit & 0xff the chunk)
        const int V = 1 << M;
        std::vector<cplx> C(size_t(V), cplx(1, 0));
        for (int j = 0; j < V; ++j)
            for (const Term &x : terms)
                if ((uint32_t(j) & x.mask) == x.mask) C[size_t(j)] *= x.v0;
        for (int ch = 0; ch < (V + 3) / 4; ++ch) {
            FOp f;
            std::memset(&f, 0, sizeof f);
            f.kind = OP_FACTOR;
            f.lbit = int32_t(uint32_t(ch) | 254u << 8);
            f.slot = -1;
            for (int e = 0; e < 4 && 4 * ch + e < V; ++e) {
                f.m[2 * e] = C[size_t(4 * ch + e)].real();
                f.m[2 * e + 1] = C[size_t(4 * ch + e)].imag();
            }
            out.push_back(f);
        }
        return;
    }
    std::vector<Term> t = terms;
    std::stable_sort(t.begin(), t.end(),
                     [](const Term &a, const Term &b) { return __builtin_popcount(a.mask) < __builtin_popcount(b.mask); });
    for (const Term &x : t) {
        FOp f;
        std::memset(&f, 0, sizeof f);
        f.kind = OP_FACTOR;
        const int code = x.sel < 0 ? 0 : (x.sel == 64 ? 255 : x.sel + 1);
        f.lbit = int32_t(x.mask | uint32_t(code) << 8);
        f.lctrl = x.ct;
        f.gctrl = x.gc;
        f.gtbit = x.sel == 64 ? x.gsel : 0;
        f.slot = -1;
        f.m[0] = x.v0.real();
        f.m[1] = x.v0.imag();
        f.m[2] = x.v1.real();
        f.m[3] = x.v1.imag();
        out.push_back(f);
    }
}

// A pass is split only when its dense ops outnumber its diagonal ones: the
// controlled phases of a QFT stage already fold into per-lane accumulators
// at one complex multiply per op and lane, and under the split each becomes
// a conditional term of a phase run instead (measured: n = 28 QFT passes
// 2.2 ms unsplit, 2.95 ms split), while a brickwork pass has no diagonal op.
bool worth_splitting(const FusedProgram &prog, const FPass &P) {
    int dense = 0, diag = 0;
    for (int o = 0; o < P.nops; ++o) {
        const FOp &x = prog.ops[size_t(P.first + o)];
        dense += x.kind == OP_DENSE;
        diag += x.kind == OP_DIAG;
    }
    return dense > 0 && dense >= diag;
}

bool has_table(const FusedProgram &prog, const FPass &P) {
    for (int o = 0; o < P.nops; ++o) {
        const FOp &x = prog.ops[size_t(P.first + o)];
        if ((x.kind == OP_DENSE || x.kind == OP_DIAG) && x.slot >= 0) return true;
    }
    return false;
}

void rewrite_pass(const FusedProgram &prog, const FPass &P, std::vector<FOp> &out) {
    const int K = P.k, M = std::min(prog.m, K);
    int rb[4] = {0, 0, 0, 0}, slot_of[32];
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

    std::vector<Item> items;
    auto phase = [&](int tb, uint64_t gt, uint32_t lc, uint64_t gc, cplx d0, cplx d1) {
        Item it;
        it.phase = true;
        it.p.tb = tb;
        it.p.gt = gt;
        it.p.lc = lc;
        it.p.gc = gc;
        it.p.d0 = d0;
        it.p.d1 = d1;
        items.push_back(it);
    };
    for (int o = 0; o < P.nops; ++o) {
        const FOp &op = prog.ops[size_t(P.first + o)];
        Item it;
        if (op.kind == OP_REMAP) {
            it.ops.push_back(op);
            items.push_back(it);
            int nrb[4];
            for (int i = 0; i < M; ++i) nrb[i] = int((op.lctrl >> (4 * i)) & 15u);
            set_layout(nrb);
            continue;
        }
        if (op.kind == OP_DENSE2) {
            it.ops.push_back(op);
            for (int r = 1; r < 4 && o + 1 < P.nops && prog.ops[size_t(P.first + o + 1)].kind == OP_CONT; ++r)
                it.ops.push_back(prog.ops[size_t(P.first + ++o)]);
            it.nset = (1u << rb[op.lbit & 0xff]) | (1u << rb[op.lbit >> 8]);
            items.push_back(it);
            continue;
        }
        if (op.kind == OP_DIAG) {
            const cplx d0(op.m[0], op.m[1]), d1(op.m[6], op.m[7]);
            // a run divides by entries (d1/d0): only entries of modulus
            // near 1 (phases) join; a projector or a scaling stays an op
            // of its own (diagonal, so it blocks no phase)
            const double a0 = std::abs(d0), a1 = std::abs(d1);
            if (a0 > 0.5 && a0 < 2.0 && a1 > 0.5 && a1 < 2.0) {
                phase(op.lbit, op.gtbit, op.lctrl, op.gctrl, d0, d1);
            } else {
                it.ops.push_back(op);
                items.push_back(it);
            }
            continue;
        }
        if (op.kind == OP_DENSE) {
            cplx r0, r1, l0, l1;
            double t;
            int form;
            const int tb = rb[op.lbit];
            if (split(op.m, r0, r1, t, form, l0, l1)) {
                phase(tb, 0, op.lctrl, op.gctrl, r0, r1);
                FOp g;
                std::memset(&g, 0, sizeof g);
                g.kind = OP_GIVENS;
                g.lbit = op.lbit | form << 8;
                g.lctrl = op.lctrl;
                g.gctrl = op.gctrl;
                g.slot = -1;
                g.m[0] = t;
                it.ops.push_back(g);
                it.nset = 1u << tb;
                items.push_back(it);
                phase(tb, 0, op.lctrl, op.gctrl, l0, l1);
                continue;
            }
        }
        // OP_DENSE kept whole, OP_PERM
        it.ops.push_back(op);
        it.nset = 1u << rb[op.lbit];
        if (op.kind == OP_PERM) {
            it.perm = true;
            it.pl = op.lctrl;
            it.pgc = op.gctrl;
        }
        items.push_back(it);
    }

    // windows: gap g lies before non-phase item g (g = N: after the last)
    std::vector<const Item *> xs;
    struct W {
        int g0, lo, hi;
        const Phase *p;
    };
    std::vector<W> win;
    for (const Item &it : items) {
        if (!it.phase) {
            xs.push_back(&it);
            continue;
        }
        win.push_back(W{int(xs.size()), int(xs.size()), int(xs.size()), &it.p});
    }
    const int N = int(xs.size());
    // the phase p, first at gap g0, moved to gap g: its components there, or
    // the farthest gap it reaches towards g
    auto move = [&](const Phase &p, int g0, int g, std::vector<Phase> &c) {
        c.assign(1, p);
        int at = g0;
        while (at < g && cross(c, *xs[size_t(at)])) ++at;
        while (at > g && cross(c, *xs[size_t(at - 1)])) --at;
        return at;
    };
    std::vector<Phase> comps;
    for (W &w : win) {
        w.lo = move(*w.p, w.g0, 0, comps);
        w.hi = move(*w.p, w.g0, N, comps);
    }
    std::stable_sort(win.begin(), win.end(), [](const W &a, const W &b) { return a.hi < b.hi; });
    // greedy stabbing: the fewest runs; run r holds windows[first[r] ..
    // first[r+1]) and may sit anywhere in [max lo, point] of its members
    std::vector<int> point, lo_max, first;
    for (size_t i = 0; i < win.size(); ++i) {
        const W &w = win[i];
        if (point.empty() || point.back() < w.lo) {
            point.push_back(w.hi);
            lo_max.push_back(w.lo);
            first.push_back(int(i));
        } else {
            lo_max.back() = std::max(lo_max.back(), w.lo);
        }
    }
    first.push_back(int(win.size()));
    // register layout at every gap
    std::vector<std::array<int, 32>> lay(size_t(N) + 1);
    set_layout(canon);
    for (int g = 0; g <= N; ++g) {
        std::copy(slot_of, slot_of + 32, lay[size_t(g)].begin());
        if (g == N) break;
        for (const FOp &op : xs[size_t(g)]->ops)
            if (op.kind == OP_REMAP) {
                int nrb[4];
                for (int i = 0; i < M; ++i) nrb[i] = int((op.lctrl >> (4 * i)) & 15u);
                set_layout(nrb);
            }
    }
    // each run at its cheapest gap (the latest on a tie)
    std::vector<std::vector<Term>> at(size_t(N) + 1);
    for (size_t r = 0; r + 1 < first.size(); ++r) {
        double best = 1e300;
        int bg = point[r];
        std::vector<Term> bt;
        for (int g = point[r]; g >= lo_max[r]; --g) {
            std::vector<Phase> run;
            for (int i = first[r]; i < first[r + 1]; ++i) {
                move(*win[size_t(i)].p, win[size_t(i)].g0, g, comps);
                run.insert(run.end(), comps.begin(), comps.end());
            }
            std::vector<Term> t = run_terms(run, lay[size_t(g)].data());
            const double c = run_cost(t, 1 << M);
            if (c < best) {
                best = c;
                bg = g;
                bt.swap(t);
            }
        }
        std::vector<Term> &dst = at[size_t(bg)];
        dst.insert(dst.end(), bt.begin(), bt.end());
    }
    set_layout(canon);
    for (int g = 0; g <= N; ++g) {
        if (!at[size_t(g)].empty()) emit_run(at[size_t(g)], M, out);
        if (g == N) break;
        for (const FOp &op : xs[size_t(g)]->ops) {
            out.push_back(op);
            if (op.kind == OP_REMAP) {
                int nrb[4];
                for (int i = 0; i < M; ++i) nrb[i] = int((op.lctrl >> (4 * i)) & 15u);
                set_layout(nrb);
            }
        }
    }
}

}  // namespace

void svi_jit_split_rotations(FusedProgram &prog, const std::vector<char> *only) {
    std::vector<FOp> out;
    out.reserve(prog.ops.size() * 2);
    for (size_t pi = 0; pi < prog.passes.size(); ++pi) {
        FPass &P = prog.passes[pi];
        const size_t first = out.size();
        if ((pi < prog.generic.size() && prog.generic[pi]) || has_table(prog, P) || (only && !(*only)[pi]))
            out.insert(out.end(), prog.ops.begin() + P.first, prog.ops.begin() + P.first + P.nops);
        else
            rewrite_pass(prog, P, out);
        P.first = int32_t(first);
        P.nops = int32_t(out.size() - first);
    }
    prog.ops.swap(out);
}

void svi_jit_transform(FusedProgram &prog) {
    const SviConfig &c = svi_config();
    if (!c.fused_jit) return;
    if (!c.fused_rotations) {
        if (c.fused_pairs) svi_jit_fuse_pairs(prog);
        return;
    }
    // each pass either takes the split or keeps composition: composition
    // reorders a pass's ops by register slot, which splits the phase windows
    std::vector<char> split(prog.passes.size()), keep(prog.passes.size());
    for (size_t p = 0; p < prog.passes.size(); ++p) {
        split[p] = worth_splitting(prog, prog.passes[p]);
        keep[p] = !split[p];
    }
    if (c.fused_pairs) svi_jit_fuse_pairs(prog, false, &keep);
    svi_jit_split_rotations(prog, &split);
}

// ---------------------------------------------------------------- host model
//
// The ops of a compiled program applied on the host in FP64, tile by tile,
// with the meaning the pass kernels give them.  It checks the host-side
// rewrites (pair fusion, rotation split, phase runs) against a plain
// simulation without a GPU; the kernels themselves are checked on the
// device.

namespace {

void model_pass(int n, const FusedProgram &prog, const FPass &P, cplx *a) {
    const int K = P.k, M = std::min(prog.m, K);
    std::vector<int> rest;
    bool in_tile[64] = {false};
    for (int i = 0; i < K; ++i) in_tile[int(P.bits[i])] = true;
    for (int b = 0; b < n; ++b)
        if (!in_tile[b]) rest.push_back(b);
    std::vector<cplx> A(size_t(1) << K);
    std::vector<uint64_t> gidx(size_t(1) << K);
    for (uint64_t w = 0; w < (uint64_t(1) << rest.size()); ++w) {
        uint64_t base = 0;
        for (size_t j = 0; j < rest.size(); ++j) base |= ((w >> j) & 1) << rest[j];
        for (uint32_t r = 0; r < (1u << K); ++r) {
            uint64_t g = base;
            for (int i = 0; i < K; ++i) g |= uint64_t((r >> i) & 1) << P.bits[i];
            gidx[r] = g;
            A[r] = a[g];
        }
        int rb[4];
        for (int i = 0; i < M; ++i) rb[i] = K - M + i;
        for (int o = 0; o < P.nops; ++o) {
            const FOp &op = prog.ops[size_t(P.first + o)];
            const bool gok = (base & op.gctrl) == op.gctrl;
            const double *m = op.m;
            switch (op.kind) {
            case OP_REMAP:
                for (int i = 0; i < M; ++i) rb[i] = int((op.lctrl >> (4 * i)) & 15u);
                break;
            case OP_DENSE:
            case OP_PERM:
            case OP_GIVENS: {
                if (!gok) break;
                const int tb = rb[op.lbit & 0xff], form = op.lbit >> 8;
                const double t = m[0];
                for (uint32_t r = 0; r < (1u << K); ++r) {
                    if (((r >> tb) & 1) || (r & op.lctrl) != op.lctrl) continue;
                    const cplx x = A[r], y = A[r | 1u << tb];
                    if (op.kind == OP_PERM) {
                        A[r] = y;
                        A[r | 1u << tb] = x;
                    } else if (op.kind == OP_DENSE) {
                        A[r] = cplx(m[0], m[1]) * x + cplx(m[2], m[3]) * y;
                        A[r | 1u << tb] = cplx(m[4], m[5]) * x + cplx(m[6], m[7]) * y;
                    } else if (form == 0) {
                        A[r] = x - t * y;
                        A[r | 1u << tb] = t * x + y;
                    } else {
                        A[r] = t * x - y;
                        A[r | 1u << tb] = x + t * y;
                    }
                }
                break;
            }
            case OP_DIAG: {
                if (!gok) break;
                const cplx d0(m[0], m[1]), d1(m[6], m[7]);
                for (uint32_t r = 0; r < (1u << K); ++r) {
                    if ((r & op.lctrl) != op.lctrl) continue;
                    const bool hi = op.lbit >= 0 ? ((r >> op.lbit) & 1) : (base & op.gtbit) != 0;
                    A[r] *= hi ? d1 : d0;
                }
                break;
            }
            case OP_DENSE2: {
                const int bl = rb[op.lbit & 0xff], bh = rb[op.lbit >> 8];
                cplx U[4][4];
                for (int rr = 0; rr < 4; ++rr)
                    for (int c = 0; c < 4; ++c) {
                        const double *mr = prog.ops[size_t(P.first + o + rr)].m;
                        U[rr][c] = cplx(mr[2 * c], mr[2 * c + 1]);
                    }
                for (uint32_t r = 0; r < (1u << K); ++r) {
                    if (((r >> bl) & 1) || ((r >> bh) & 1)) continue;
                    const uint32_t idx[4] = {r, r | 1u << bl, r | 1u << bh, r | 1u << bl | 1u << bh};
                    cplx x[4], y[4];
                    for (int c = 0; c < 4; ++c) x[c] = A[idx[c]];
                    for (int rr = 0; rr < 4; ++rr) {
                        y[rr] = 0.0;
                        for (int c = 0; c < 4; ++c) y[rr] += U[rr][c] * x[c];
                    }
                    for (int c = 0; c < 4; ++c) A[idx[c]] = y[c];
                }
                break;
            }
            case OP_FACTOR: {
                if (!gok) break;
                const int code = (op.lbit >> 8) & 0xff;
                if (code == 254) {
                    // entries 4 c .. 4 c + 3 of the run's table, by register index
                    const int ch = op.lbit & 0xff;
                    for (uint32_t r = 0; r < (1u << K); ++r) {
                        int j = 0;
                        for (int i = 0; i < M; ++i) j |= int((r >> rb[i]) & 1) << i;
                        if (j / 4 == ch) A[r] *= cplx(m[2 * (j % 4)], m[2 * (j % 4) + 1]);
                    }
                    break;
                }
                uint32_t lm = 0;
                for (int i = 0; i < M; ++i)
                    if ((op.lbit >> i) & 1) lm |= 1u << rb[i];
                const cplx v0(m[0], m[1]), v1(m[2], m[3]);
                for (uint32_t r = 0; r < (1u << K); ++r) {
                    if ((r & lm) != lm || (r & op.lctrl) != op.lctrl) continue;
                    bool hi = false;
                    if (code == 255)
                        hi = (base & op.gtbit) != 0;
                    else if (code > 0)
                        hi = (r >> (code - 1)) & 1;
                    A[r] *= hi ? v1 : v0;
                }
                break;
            }
            default:
                break;  // OP_CONT: rows of the OP_DENSE2 before it
            }
        }
        for (uint32_t r = 0; r < (1u << K); ++r) a[gidx[r]] = A[r];
    }
}

}  // namespace

extern "C" int sv_model_fused(int n, int dtype, const sv_gate *gates, int64_t ng, double *amps) {
    if (n < 1 || n > 24 || (dtype != SV_C64 && dtype != SV_C128) || ng < 0 || (ng > 0 && !gates) || !amps)
        return SV_EINVAL;
    std::vector<PreparedGate> prep;
    int rc = svi_prepare(n, gates, ng, prep, nullptr);
    if (rc != SV_OK) return rc;
    FusedProgram prog;
    rc = svi_fused_compile(n, dtype, prep.data(), ng, prog);
    if (rc != SV_OK) return rc;
    svi_jit_transform(prog);
    cplx *a = reinterpret_cast<cplx *>(amps);
    for (const FusedProgram::Item &it : prog.items) {
        if (!it.swap) {
            model_pass(n, prog, prog.passes[size_t(it.pass)], a);
            continue;
        }
        const int b1 = n - 1 - it.q1, b2 = n - 1 - it.q2;
        for (uint64_t j = 0; j < (uint64_t(1) << n); ++j)
            if (((j >> b1) & 1) && !((j >> b2) & 1)) std::swap(a[j], a[j ^ (uint64_t(1) << b1) ^ (uint64_t(1) << b2)]);
    }
    return SV_OK;
}
