// Fused multi-gate passes: one HBM sweep applies a whole run of gates.
//
// The per-gate path (sec. 2.2.1/2.2.2 applied one evolution step at a time,
// as the paper's simulator does) reads and writes the full register for
// every gate.  Here a pass loads a tile of 2^K amplitudes into LDS, applies
// every gate scheduled into the pass, and writes the tile back once.
//
// Tile.  The tile bits are the nlow lowest index bits (contiguous runs of
// 2^nlow amplitudes in HBM, for coalesced loads) plus up to K - nlow chosen
// higher bits.  Workgroup tau owns the 2^K amplitudes whose non-tile bits
// spell tau.  Within the tile, local index r maps to the global index by
// depositing r's bits on the tile bit positions.
//
// Registers.  The 2^K amplitudes of a tile live in registers: each of the
// 2^(K-M) threads holds 2^M of them.  A layout names M local bits as
// "register bits"; thread t's register j holds local index
// deposit(t, other bits) | deposit(j, register bits).  A gate whose target is
// a register bit is applied inside each thread with no LDS traffic and no
// barrier; a diagonal gate is applied in registers whatever its bits.  Only
// a change of register bits (OP_REMAP) goes through LDS: every thread writes
// its amplitudes, a barrier, every thread reads its new ones.  LDS addresses
// are XOR-swizzled so that strided layouts do not pile onto one bank.  Each
// tile is loaded and stored in the canonical layout (register bits = the top
// M local bits) so consecutive lanes touch consecutive amplitudes.
//
// Which gates fit a pass.
//   - A non-diagonal gate needs its target bit in the tile (its pairs must
//     lie inside one tile); its controls may be anywhere: a control outside
//     the tile has one value for the whole tile, so it is a per-workgroup
//     uniform test (sec. 2.2.2 rows with a control bit 0 are identity rows).
//   - A diagonal gate (Z, R_k, controlled phases) is an elementwise scaling,
//     so it fits every pass: an out-of-tile target bit again has one value
//     per tile.
// Scheduling.  Gates are scanned in order; a gate joins the pass unless it
// must stay after an earlier deferred gate.  Two gates may be reordered
// unless they share a qubit on which either acts non-diagonally (as the
// target of a non-diagonal matrix): gates that are block diagonal over all
// shared qubits commute.  A deferred gate blocks its qubits for the rest of
// the scan; SWAP gates end the pass and run as their own permutation kernel.
// Inside a pass the same rule splits the gates into register-bit segments.
#include <algorithm>
#include <cstring>
#include <vector>

#include "device_common.h"
#include "fused.h"

using namespace svd;

namespace {

template <int K>
__device__ __forceinline__ uint64_t tile_index(uint64_t base, uint32_t r, uint32_t lowmask, int nlow,
                                               const int8_t *bits) {
    uint64_t g = base | (r & lowmask);
#pragma unroll
    for (int i = 0; i < K; ++i)
        if (i >= nlow) g |= uint64_t((r >> i) & 1) << bits[i];
    return g;
}

// XOR swizzle of an LDS element index: folds the bits above each 256-byte
// bank window onto the bank-selecting low bits.
template <typename T>
__device__ __forceinline__ uint32_t swz(uint32_t r) {
    constexpr int SB = sizeof(T) == 16 ? 4 : 5;
    return r ^ (((r >> SB) ^ (r >> (2 * SB))) & ((1u << SB) - 1));
}

// Workgroup barrier that orders LDS accesses only.  __syncthreads() is a
// fence over all address spaces, which would also wait for outstanding HBM
// accesses; the exchanges here only communicate through LDS.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Local-index offset of register j: the register-bit masks of the set bits
// of j (j is a compile-time constant after unrolling, so this folds to a few
// ORs of uniform values).
template <int M>
__device__ __forceinline__ uint32_t reg_off(const uint32_t (&rbit)[M], int j) {
    uint32_t x = 0;
#pragma unroll
    for (int i = 0; i < M; ++i)
        if ((j >> i) & 1) x |= rbit[i];
    return x;
}

// A 2x2 complex matrix held in named scalars (an array indexed through a
// runtime select would be placed in scratch memory).
template <typename R>
struct Mat8 {
    R a, b, c, d, e, f, g, h;  // u11re u11im u12re u12im u21re u21im u22re u22im
};

template <typename T, typename R>
__device__ __forceinline__ T row_mac(R ur, R ui, R vr, R vi, T x, T y) {
    T r;
    r.x = ur * x.x - ui * x.y + vr * y.x - vi * y.y;
    r.y = ur * x.y + ui * x.x + vr * y.y + vi * y.x;
    return r;
}

// Register pairs (j, j | 2^S) of a gate whose target is register slot S.
// MODE 0: dense, no control inside the tile; 1: dense with in-tile
// controls; 2: exact NOT, no in-tile control (a plain exchange); 3: exact
// NOT with in-tile controls.  The NOT paths move values without arithmetic,
// so permutations stay bit-exact.
template <typename T, typename R, int M, int S, int MODE>
__device__ __forceinline__ void reg_pairs(T (&v)[1 << M], const uint32_t (&rbit)[M], uint32_t tpart,
                                          uint32_t lctrl, const Mat8<R> &m) {
#pragma unroll
    for (int j = 0; j < (1 << M); ++j) {
        if ((j >> S) & 1) continue;
        const int jj = j | (1 << S);
        const T x = v[j], y = v[jj];
        if (MODE == 0) {
            v[j] = row_mac<T, R>(m.a, m.b, m.c, m.d, x, y);
            v[jj] = row_mac<T, R>(m.e, m.f, m.g, m.h, x, y);
        } else if (MODE == 2) {
            v[j] = y;
            v[jj] = x;
        } else {
            const bool ok = ((tpart | reg_off<M>(rbit, j)) & lctrl) == lctrl;
            T nx, ny;
            if (MODE == 1) {
                nx = row_mac<T, R>(m.a, m.b, m.c, m.d, x, y);
                ny = row_mac<T, R>(m.e, m.f, m.g, m.h, x, y);
            } else {
                nx = y;
                ny = x;
            }
            v[j] = ok ? nx : x;
            v[jj] = ok ? ny : y;
        }
    }
}

template <typename T, typename R, int M, int S>
__device__ __forceinline__ void reg_slot(int mode, T (&v)[1 << M], const uint32_t (&rbit)[M], uint32_t tpart,
                                         uint32_t lctrl, const Mat8<R> &m) {
    switch (mode) {
    case 0: reg_pairs<T, R, M, S, 0>(v, rbit, tpart, lctrl, m); break;
    case 1: reg_pairs<T, R, M, S, 1>(v, rbit, tpart, lctrl, m); break;
    case 2: reg_pairs<T, R, M, S, 2>(v, rbit, tpart, lctrl, m); break;
    default: reg_pairs<T, R, M, S, 3>(v, rbit, tpart, lctrl, m); break;
    }
}

template <typename T, typename R, int M>
__device__ __forceinline__ void reg_gate(int slot, int mode, T (&v)[1 << M], const uint32_t (&rbit)[M],
                                         uint32_t tpart, uint32_t lctrl, const Mat8<R> &m) {
    switch (slot) {
    case 0: reg_slot<T, R, M, 0>(mode, v, rbit, tpart, lctrl, m); break;
    case 1: if constexpr (M > 1) reg_slot<T, R, M, 1>(mode, v, rbit, tpart, lctrl, m); break;
    case 2: if constexpr (M > 2) reg_slot<T, R, M, 2>(mode, v, rbit, tpart, lctrl, m); break;
    case 3: if constexpr (M > 3) reg_slot<T, R, M, 3>(mode, v, rbit, tpart, lctrl, m); break;
    case 4: if constexpr (M > 4) reg_slot<T, R, M, 4>(mode, v, rbit, tpart, lctrl, m); break;
    default: break;
    }
}

// Layout: register bits rb[0..M-1] (local positions, 4 bits each in
// packed); thread bits are the other K - M local bits in ascending order.
template <int K, int M>
__device__ __forceinline__ void set_layout(uint32_t packed, int t, uint32_t &tpart, uint32_t (&rbit)[M]) {
    uint32_t rbmask = 0;
#pragma unroll
    for (int i = 0; i < M; ++i) {
        rbit[i] = 1u << ((packed >> (4 * i)) & 15);
        rbmask |= rbit[i];
    }
    uint32_t tp = 0;
    int src = 0;
#pragma unroll
    for (int b = 0; b < K; ++b) {
        if ((rbmask >> b) & 1) continue;
        tp |= uint32_t((t >> src) & 1) << b;
        ++src;
    }
    tpart = tp;
}

// Workgroup w handles tile (w mod 2^tile_bits) of register (w >> tile_bits):
// a batch of registers is stored back to back, 2^n amplitudes each, and the
// per-register matrices of table-driven ops sit in rows of nslots matrices.
template <typename T, int K, int M>
__global__ __launch_bounds__(1 << (K - M)) void k_fused(T *__restrict__ a, const FPass *__restrict__ pass,
                                                        const FOp *__restrict__ ops,
                                                        const typename RealOf<T>::type *__restrict__ table,
                                                        uint32_t nslots, int tile_bits, int n) {
    using R = typename RealOf<T>::type;
    constexpr int V = 1 << M;
    constexpr uint32_t TILE = 1u << K;
    __shared__ T lds[TILE];
    const FPass P = *pass;
    const int t = threadIdx.x;
    const uint32_t lowmask = (1u << P.nlow) - 1;
    const uint64_t reg = uint64_t(blockIdx.x) >> tile_bits;
    a += reg << n;
    const R *trow = table ? table + reg * uint64_t(nslots) * 8 : nullptr;
    uint64_t base = uint64_t(blockIdx.x) & ((uint64_t(1) << tile_bits) - 1);
#pragma unroll
    for (int i = 0; i < K; ++i) base = insert_zero(base, P.bits[i]);

    // canonical layout: thread bits are the low K - M local bits
    uint32_t tpart = uint32_t(t);
    uint32_t rbit[M];
#pragma unroll
    for (int i = 0; i < M; ++i) rbit[i] = 1u << (K - M + i);
    T v[V];
#pragma unroll
    for (int j = 0; j < V; ++j)
        v[j] = ldnt(a + tile_index<K>(base, tpart | (uint32_t(j) << (K - M)), lowmask, P.nlow, P.bits));

    bool lds_live = false;
    // op descriptors are uniform (scalar loads); the op is interpreted at run
    // time, which the specialised kernels of jit.hip avoid
    const FOp *op = ops + P.first;
    for (int o = 0; o < P.nops; ++o) {
        const FOp &cur = op[o];
        const int kind = cur.kind;
        if (kind == OP_REMAP) {
            if (lds_live) lds_barrier();
#pragma unroll
            for (int j = 0; j < V; ++j) lds[swz<T>(tpart | reg_off<M>(rbit, j))] = v[j];
            lds_barrier();
            set_layout<K, M>(cur.lctrl, t, tpart, rbit);
#pragma unroll
            for (int j = 0; j < V; ++j) v[j] = lds[swz<T>(tpart | reg_off<M>(rbit, j))];
            lds_live = true;
        } else if ((base & cur.gctrl) == cur.gctrl) {  // uniform over the workgroup
            Mat8<R> m;
            if (cur.slot >= 0) {
                const R *tm = trow + size_t(cur.slot) * 8;
                m.a = tm[0];
                m.b = tm[1];
                m.c = tm[2];
                m.d = tm[3];
                m.e = tm[4];
                m.f = tm[5];
                m.g = tm[6];
                m.h = tm[7];
            } else {
                m.a = R(cur.m[0]);
                m.b = R(cur.m[1]);
                m.c = R(cur.m[2]);
                m.d = R(cur.m[3]);
                m.e = R(cur.m[4]);
                m.f = R(cur.m[5]);
                m.g = R(cur.m[6]);
                m.h = R(cur.m[7]);
            }
            const uint32_t lctrl = cur.lctrl;
            if (kind == OP_DIAG) {
                const int lb = cur.lbit;
                if (lb >= 0) {
#pragma unroll
                    for (int j = 0; j < V; ++j) {
                        const uint32_t r = tpart | reg_off<M>(rbit, j);
                        if ((r & lctrl) != lctrl) continue;
                        const bool hi = (r >> lb) & 1;
                        const R fr = hi ? m.g : m.a, fi = hi ? m.h : m.b;
                        v[j] = cscale<T, R>(fr, fi, v[j]);
                    }
                } else {
                    const bool hi = (base & cur.gtbit) != 0;
                    const R fr = hi ? m.g : m.a, fi = hi ? m.h : m.b;
                    if (!(fr == R(1) && fi == R(0))) {
#pragma unroll
                        for (int j = 0; j < V; ++j) {
                            const uint32_t r = tpart | reg_off<M>(rbit, j);
                            if ((r & lctrl) != lctrl) continue;
                            v[j] = cscale<T, R>(fr, fi, v[j]);
                        }
                    }
                }
            } else {
                const int mode = (kind == OP_PERM ? 2 : 0) + (lctrl != 0 ? 1 : 0);
                reg_gate<T, R, M>(cur.lbit, mode, v, rbit, tpart, lctrl, m);
            }
        }
    }
    // the planner ends every pass in the canonical layout
#pragma unroll
    for (int j = 0; j < V; ++j)
        stnt(v[j], a + tile_index<K>(base, tpart | reg_off<M>(rbit, j), lowmask, P.nlow, P.bits));
}

// ------------------------------------------------------------------ planner

enum Mode : uint8_t { M_NONE = 0, M_DIAG = 1, M_FULL = 2 };

struct PlannedPass {
    std::vector<int> bits;  // ascending tile bits
    int nlow = 0;
    std::vector<FOp> ops;
    std::vector<int64_t> gate_ids;  // gates of the pass, in execution order
};
struct Step {
    bool is_swap;
    int q1, q2;
    PlannedPass pass;
};

inline bool conflicts(const uint8_t *blk, int bit, Mode m) {
    return blk[bit] == M_FULL || (blk[bit] == M_DIAG && m == M_FULL);
}
inline void block(uint8_t *blk, int bit, Mode m) {
    if (blk[bit] < m) blk[bit] = m;
}

// True if gate x may run before every gate already blocking bits in blk.
inline bool free_of_blocks(const uint8_t *blk, int n, const PreparedGate &x) {
    const int tb = n - 1 - x.q;
    if (conflicts(blk, tb, x.cls == GC_DIAG ? M_DIAG : M_FULL)) return false;
    for (uint64_t c = x.ctrl; c; c &= c - 1)
        if (conflicts(blk, __builtin_ctzll(c), M_DIAG)) return false;
    return true;
}
inline void block_gate(uint8_t *blk, int n, const PreparedGate &x) {
    block(blk, n - 1 - x.q, x.cls == GC_DIAG ? M_DIAG : M_FULL);
    for (uint64_t c = x.ctrl; c; c &= c - 1) block(blk, __builtin_ctzll(c), M_DIAG);
}

// Splits the gates of one pass into register-bit segments (see the kernel)
// and emits the op list: REMAP ops between segments, a final REMAP back to
// the canonical layout (register bits K-M..K-1) when needed.
void build_pass_ops(int n, const PreparedGate *g, PlannedPass &p, int M) {
    const int K = int(p.bits.size());
    int local[64];
    bool in_tile[64] = {false};
    for (int i = 0; i < K; ++i) {
        local[p.bits[size_t(i)]] = i;
        in_tile[p.bits[size_t(i)]] = true;
    }
    uint32_t canon = 0;
    for (int i = 0; i < M; ++i) canon |= uint32_t(K - M + i) << (4 * i);
    auto make_op = [&](const PreparedGate &x, int slot) {
        FOp op;
        std::memset(&op, 0, sizeof op);
        const int tb = n - 1 - x.q;
        op.kind = x.cls == GC_DIAG ? OP_DIAG : (x.cls == GC_PERM ? OP_PERM : OP_DENSE);
        if (op.kind == OP_DIAG) {
            op.lbit = in_tile[tb] ? local[tb] : -1;
            op.gtbit = in_tile[tb] ? 0 : (uint64_t(1) << tb);
        } else {
            op.lbit = slot;
        }
        for (uint64_t c = x.ctrl; c; c &= c - 1) {
            const int cb = __builtin_ctzll(c);
            if (in_tile[cb])
                op.lctrl |= 1u << local[cb];
            else
                op.gctrl |= uint64_t(1) << cb;
        }
        for (int j = 0; j < 8; ++j) op.m[j] = x.U[j];
        op.slot = x.slot;
        return op;
    };
    std::vector<int64_t> rem = p.gate_ids, order;
    p.ops.clear();
    uint32_t cur = canon;
    bool first = true;
    while (!rem.empty()) {
        // register set of this segment; the first one starts from the
        // canonical layout so that its gates need no exchange
        int regs[8];
        int nreg = 0;
        if (first)
            for (int i = 0; i < M; ++i) regs[nreg++] = K - M + i;
        uint8_t blk[64] = {0};
        std::vector<int64_t> take, deferred;
        for (int64_t id : rem) {
            const PreparedGate &x = g[id];
            bool ok = free_of_blocks(blk, n, x);
            int slot = -1;
            if (ok && x.cls != GC_DIAG) {
                const int lb = local[n - 1 - x.q];
                for (int i = 0; i < nreg; ++i)
                    if (regs[i] == lb) slot = i;
                if (slot < 0) {
                    if (nreg < M) {
                        regs[nreg] = lb;
                        slot = nreg++;
                    } else {
                        ok = false;
                    }
                }
            }
            if (ok) {
                take.push_back(id);
            } else {
                deferred.push_back(id);
                block_gate(blk, n, x);
            }
        }
        if (!take.empty()) {
            // fill the register set up to M bits, keeping slots of taken gates
            for (int b = 0; b < K && nreg < M; ++b) {
                bool used = false;
                for (int i = 0; i < nreg; ++i) used |= regs[i] == b;
                if (!used) regs[nreg++] = b;
            }
            uint32_t packed = 0;
            for (int i = 0; i < M; ++i) packed |= uint32_t(regs[i]) << (4 * i);
            if (packed != cur) {
                FOp r;
                std::memset(&r, 0, sizeof r);
                r.kind = OP_REMAP;
                r.lctrl = packed;
                p.ops.push_back(r);
                cur = packed;
            }
            for (int64_t id : take) {
                const PreparedGate &x = g[id];
                int slot = -1;
                if (x.cls != GC_DIAG) {
                    const int lb = local[n - 1 - x.q];
                    for (int i = 0; i < M; ++i)
                        if (regs[i] == lb) slot = i;
                }
                p.ops.push_back(make_op(x, slot));
                order.push_back(id);
            }
        }
        first = false;
        rem.swap(deferred);
    }
    if (cur != canon) {
        FOp r;
        std::memset(&r, 0, sizeof r);
        r.kind = OP_REMAP;
        r.lctrl = canon;
        p.ops.push_back(r);
    }
    p.gate_ids.swap(order);
}

std::vector<Step> plan(int n, const PreparedGate *g, int64_t ng, int K, int M, int nlow_req, int max_ops,
                       bool search) {
    std::vector<Step> steps;
    K = std::min(K, n);
    M = std::min(M, K);
    const int nlow = std::min(nlow_req, K);
    std::vector<int64_t> rem(static_cast<size_t>(ng));
    for (int64_t i = 0; i < ng; ++i) rem[size_t(i)] = i;
    size_t head = 0;  // rem[head..] still to place
    while (head < rem.size()) {
        const PreparedGate &g0 = g[rem[head]];
        if (g0.kind == SV_G_SWAP) {
            Step st;
            st.is_swap = true;
            st.q1 = g0.q;
            st.q2 = g0.q2;
            st.pass.gate_ids.push_back(rem[head]);
            steps.push_back(std::move(st));
            ++head;
            continue;
        }
        // One scan in program order: a gate joins unless it must follow a
        // deferred gate, or (non-diagonal) its target bit is outside the
        // tile and no slot is left.  fixed = true: the tile is given and
        // takes no new bits.  Returns the next unscanned index.
        auto scan = [&](bool *in_tile, int &free_slots, bool fixed, std::vector<int64_t> &sched,
                        std::vector<int64_t> &deferred) {
            uint8_t blk[64] = {0};
            size_t i = head;
            for (; i < rem.size(); ++i) {
                const PreparedGate &x = g[rem[i]];
                if (x.kind == SV_G_SWAP) {
                    // a permutation of two qubits: everything after it on those
                    // qubits waits; other gates may still join this pass
                    deferred.push_back(rem[i]);
                    block(blk, n - 1 - x.q, M_FULL);
                    block(blk, n - 1 - x.q2, M_FULL);
                    continue;
                }
                const int tb = n - 1 - x.q;
                bool ok = free_of_blocks(blk, n, x);
                if (ok && int(sched.size()) >= max_ops) ok = false;
                if (ok && x.cls != GC_DIAG && !in_tile[tb]) {
                    if (!fixed && free_slots > 0) {
                        in_tile[tb] = true;
                        --free_slots;
                    } else {
                        ok = false;
                    }
                }
                if (ok) {
                    sched.push_back(rem[i]);
                } else {
                    deferred.push_back(rem[i]);
                    block_gate(blk, n, x);
                    // stop scanning once every qubit is fully blocked
                    bool all = true;
                    for (int b = 0; b < n && all; ++b) all = blk[b] == M_FULL;
                    if (all) return i + 1;
                }
            }
            return i;
        };
        auto work = [&](const std::vector<int64_t> &sched) {
            double w = 0.0;
            for (int64_t id : sched) w += g[id].cls == GC_DIAG ? 0.25 : (g[id].cls == GC_PERM ? 0.5 : 1.0);
            return w;
        };
        bool in_tile[64] = {false};
        for (int b = 0; b < nlow; ++b) in_tile[b] = true;
        int free_slots = K - nlow;
        std::vector<int64_t> sched, deferred;
        size_t i = scan(in_tile, free_slots, false, sched, deferred);
        if (search && free_slots == 0) {
            // tiles of contiguous qubits can advance a light cone over
            // several layers: try every window of the free slots' width
            // above the low bits and keep the one that schedules the most
            const int w = K - nlow;
            double best = work(sched);
            for (int lo = nlow; lo + w <= n; ++lo) {
                bool t2[64] = {false};
                for (int b = 0; b < nlow; ++b) t2[b] = true;
                for (int b = lo; b < lo + w; ++b) t2[b] = true;
                int fs = 0;
                std::vector<int64_t> s2, d2;
                const size_t i2 = scan(t2, fs, true, s2, d2);
                const double sc = work(s2);
                if (sc > best) {
                    best = sc;
                    std::memcpy(in_tile, t2, sizeof t2);
                    sched.swap(s2);
                    deferred.swap(d2);
                    i = i2;
                }
            }
        }
        // unscanned gates stay queued after the deferred ones, in order
        for (; i < rem.size(); ++i) deferred.push_back(rem[i]);
        // fill unused slots with the lowest free bits (longer HBM runs)
        for (int b = 0; b < n && free_slots > 0; ++b)
            if (!in_tile[b]) {
                in_tile[b] = true;
                --free_slots;
            }
        Step st;
        st.is_swap = false;
        PlannedPass &p = st.pass;
        for (int b = 0; b < n; ++b)
            if (in_tile[b]) p.bits.push_back(b);
        int nl = 0;
        while (nl < int(p.bits.size()) && p.bits[size_t(nl)] == nl) ++nl;
        p.nlow = nl;
        p.gate_ids = sched;
        build_pass_ops(n, g, p, M);
        steps.push_back(std::move(st));
        rem.erase(rem.begin() + std::ptrdiff_t(head), rem.end());
        rem.insert(rem.end(), deferred.begin(), deferred.end());
    }
    return steps;
}

template <typename T, int K>
hipError_t launch_pass(const FusedLaunch &L, const FPass *dpass, const FOp *dops) {
    using R = typename RealOf<T>::type;
    constexpr int MDEF = 4;
    constexpr int M = K < MDEF ? K : MDEF;
    constexpr int NT = 1 << (K - M);
    const int tile_bits = L.n - K;
    const uint64_t grid = L.nregs << tile_bits;
    if (grid == 0 || grid > 0x7fffffffull) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_fused<T, K, M>), dim3(unsigned(grid)), dim3(NT), 0, L.stream, static_cast<T *>(L.state),
                       dpass, dops, static_cast<const R *>(L.table), L.nslots, tile_bits, L.n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pass_k(const FusedLaunch &L, int K, const FPass *dpass, const FOp *dops) {
    switch (K) {
    case 1: return launch_pass<T, 1>(L, dpass, dops);
    case 2: return launch_pass<T, 2>(L, dpass, dops);
    case 3: return launch_pass<T, 3>(L, dpass, dops);
    case 4: return launch_pass<T, 4>(L, dpass, dops);
    case 5: return launch_pass<T, 5>(L, dpass, dops);
    case 6: return launch_pass<T, 6>(L, dpass, dops);
    case 7: return launch_pass<T, 7>(L, dpass, dops);
    case 8: return launch_pass<T, 8>(L, dpass, dops);
    case 9: return launch_pass<T, 9>(L, dpass, dops);
    case 10: return launch_pass<T, 10>(L, dpass, dops);
    case 11: return launch_pass<T, 11>(L, dpass, dops);
    case 12: return launch_pass<T, 12>(L, dpass, dops);
    case 13:
        if constexpr (sizeof(T) == 8) return launch_pass<T, 13>(L, dpass, dops);
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

// Register bits per thread (16 amplitudes; tiles smaller than that use K).
inline int reg_bits_for(int) { return 4; }

}  // namespace

// Device and pinned staging memory for pass descriptors, grown on demand.
struct FusedBuffers {
    void *dev = nullptr;
    void *host = nullptr;
    size_t cap = 0;
    hipEvent_t uploaded = nullptr;  // host buffer may be rewritten once this completes
    hipEvent_t done = nullptr;      // last pass of the previous run (device buffer in use until then)
};

void svi_release_fused(sv_state *s) {
    if (!s->fused) return;
    FusedBuffers *f = s->fused;
    if (f->uploaded) {
        (void)hipEventSynchronize(f->uploaded);
        (void)hipEventDestroy(f->uploaded);
    }
    if (f->done) {
        (void)hipEventSynchronize(f->done);
        (void)hipEventDestroy(f->done);
    }
    if (f->dev) (void)hipFree(f->dev);
    if (f->host) (void)hipHostFree(f->host);
    delete f;
    s->fused = nullptr;
}

int svi_fused_compile(int n, int dtype, const PreparedGate *gates, int64_t ng, FusedProgram &out) {
    const SviConfig &cfg = svi_config();
    const int K = dtype == SV_C128 ? cfg.fused_tile_bits_c128 : cfg.fused_tile_bits_c64;
    // the generic kernel is built for 4 register bits; specialised kernels
    // take any count
    const int m = cfg.fused_jit ? cfg.fused_reg_bits : reg_bits_for(dtype);
    const std::vector<Step> steps =
        plan(n, gates, ng, K, m, cfg.fused_low_bits, cfg.fused_max_ops, cfg.fused_plan_search != 0);
    out = FusedProgram();
    out.m = m;
    for (const Step &st : steps) {
        FusedProgram::Item it;
        it.swap = st.is_swap;
        it.q1 = st.q1;
        it.q2 = st.q2;
        it.pass = -1;
        if (!st.is_swap) {
            FPass P;
            std::memset(&P, 0, sizeof P);
            P.k = int32_t(st.pass.bits.size());
            P.nlow = st.pass.nlow;
            P.first = int32_t(out.ops.size());
            P.nops = int32_t(st.pass.ops.size());
            for (size_t j = 0; j < st.pass.bits.size(); ++j) P.bits[j] = int8_t(st.pass.bits[j]);
            it.pass = int(out.passes.size());
            out.passes.push_back(P);
            out.ops.insert(out.ops.end(), st.pass.ops.begin(), st.pass.ops.end());
        }
        for (int64_t id : st.pass.gate_ids) {
            out.order.push_back(id);
            out.pass_of.push_back(it.pass);
        }
        out.items.push_back(it);
    }
    out.generic.assign(out.passes.size(), 0);
    if (cfg.fused_jit && m == reg_bits_for(dtype))
        for (size_t p = 0; p < out.passes.size(); ++p) out.generic[p] = out.passes[p].nops > cfg.fused_jit_max_ops;
    return int64_t(out.order.size()) == ng ? SV_OK : SV_EDEVICE;
}

hipError_t svi_fused_launch_pass(const FusedLaunch &L, int k, const FPass *dpass, const FOp *dops) {
    return L.dtype == SV_C128 ? launch_pass_k<c128>(L, k, dpass, dops) : launch_pass_k<c64>(L, k, dpass, dops);
}

int svi_run_fused(sv_state *s, const PreparedGate *gates, int64_t ng, bool prof) {
    FusedProgram prog;
    int rc = svi_fused_compile(s->n, s->dtype, gates, ng, prog);
    if (rc != SV_OK) return rc;
    svi_jit_transform(prog);

    // pack descriptors: FPass array, then FOp array
    const size_t npass = prog.passes.size(), nops = prog.ops.size();
    const size_t pass_bytes = (npass * sizeof(FPass) + 255) & ~size_t(255);
    const size_t bytes = pass_bytes + nops * sizeof(FOp) + 256;
    if (!s->fused) s->fused = new FusedBuffers();
    FusedBuffers *f = s->fused;
    if (f->uploaded) {
        // the previous upload must have left the pinned buffer before reuse
        if (hipEventSynchronize(f->uploaded) != hipSuccess) return SV_EDEVICE;
    } else if (hipEventCreateWithFlags(&f->uploaded, hipEventDisableTiming) != hipSuccess ||
               hipEventCreateWithFlags(&f->done, hipEventDisableTiming) != hipSuccess) {
        return SV_EDEVICE;
    } else if (hipEventRecord(f->done, s->stream) != hipSuccess) {
        return SV_EDEVICE;
    }
    // the previous run may have used another stream: its passes must finish
    // reading the device descriptors before this run's upload overwrites them
    if (hipStreamWaitEvent(s->stream, f->done, 0) != hipSuccess) return SV_EDEVICE;
    if (bytes > f->cap) {
        // kernels of an earlier call may still read the old device buffer
        if (f->dev && hipStreamSynchronize(s->stream) != hipSuccess) return SV_EDEVICE;
        if (f->dev) (void)hipFree(f->dev);
        if (f->host) (void)hipHostFree(f->host);
        f->dev = f->host = nullptr;
        f->cap = 0;
        size_t cap = std::max<size_t>(bytes, 64 * 1024);
        if (hipMalloc(&f->dev, cap) != hipSuccess) return SV_ENOMEM;
        if (hipHostMalloc(&f->host, cap, hipHostMallocDefault) != hipSuccess) return SV_ENOMEM;
        f->cap = cap;
    }
    if (npass) std::memcpy(f->host, prog.passes.data(), npass * sizeof(FPass));
    if (nops) std::memcpy(static_cast<char *>(f->host) + pass_bytes, prog.ops.data(), nops * sizeof(FOp));
    if (hipMemcpyAsync(f->dev, f->host, bytes - 256, hipMemcpyHostToDevice, s->stream) != hipSuccess)
        return SV_EDEVICE;
    if (hipEventRecord(f->uploaded, s->stream) != hipSuccess) return SV_EDEVICE;

    std::vector<hipFunction_t> jit;
    if (svi_config().fused_jit) {
        rc = svi_jit_prepare(s->device, s->dtype, prog, jit);
        if (rc != SV_OK) return rc;
    }
    const FPass *dp = static_cast<const FPass *>(f->dev);
    const FOp *dops = reinterpret_cast<const FOp *>(static_cast<char *>(f->dev) + pass_bytes);
    FusedLaunch L;
    L.state = s->d;
    L.n = s->n;
    L.dtype = s->dtype;
    L.stream = s->stream;
    L.table = nullptr;
    L.nslots = 0;
    L.nregs = 1;
    const bool bitperm = svi_config().swap_runs != 0;
    for (size_t ii = 0; ii < prog.items.size(); ++ii) {
        const FusedProgram::Item &it = prog.items[ii];
        hipError_t e;
        if (it.swap && bitperm) {
            // a run of swaps whose product is an involution on the index
            // bits moves every amplitude once (one permutation pass)
            size_t jj = ii;
            int f[64];
            for (int b = 0; b < s->n; ++b) f[b] = b;
            while (jj < prog.items.size() && prog.items[jj].swap) {
                const int b1 = s->n - 1 - prog.items[jj].q1, b2 = s->n - 1 - prog.items[jj].q2;
                int g[64];
                for (int b = 0; b < s->n; ++b) g[b] = f[b == b1 ? b2 : (b == b2 ? b1 : b)];
                for (int b = 0; b < s->n; ++b) f[b] = g[b];
                ++jj;
            }
            bool invol = jj - ii >= 2;
            for (int b = 0; b < s->n && invol; ++b) invol = f[f[b]] == b;
            if (invol) {
                const int slot = svi_prof_begin(s, prof, STEP_SWAP);
                e = svi_launch_bitperm(s, f);
                svi_prof_end(s, slot);
                if (e != hipSuccess) return svi_fail("sv_run (bit permutation)", e);
                ii = jj - 1;
                continue;
            }
        }
        const int slot = svi_prof_begin(s, prof, it.swap ? STEP_SWAP : STEP_FUSED_PASS);
        if (it.swap) {
            e = svi_launch_swap(s, it.q1, it.q2);
        } else {
            const int k = prog.passes[size_t(it.pass)].k;
            e = (jit.empty() || !jit[size_t(it.pass)])
                    ? svi_fused_launch_pass(L, k, dp + it.pass, dops)
                    : svi_jit_launch(jit[size_t(it.pass)], L, k, std::min(prog.m, k), dp + it.pass, dops);
        }
        svi_prof_end(s, slot);
        if (e != hipSuccess) return svi_status_from_hip(e);
    }
    if (hipEventRecord(f->done, s->stream) != hipSuccess) return SV_EDEVICE;
    return SV_OK;
}

extern "C" int sv_plan_fused(int n, int dtype, const sv_gate *gates, int64_t ng, int64_t *order, int32_t *pass_of,
                             uint64_t *tile_mask, int64_t *npasses) {
    if (n < 1 || n > SV_MAX_QUBITS || (dtype != SV_C64 && dtype != SV_C128) || ng < 0 || (ng > 0 && !gates) ||
        !npasses)
        return SV_EINVAL;
    std::vector<PreparedGate> prep;
    int rc = svi_prepare(n, gates, ng, prep, nullptr);
    if (rc != SV_OK) return rc;
    FusedProgram prog;
    rc = svi_fused_compile(n, dtype, prep.data(), ng, prog);
    if (rc != SV_OK) return rc;
    for (size_t i = 0; i < prog.order.size(); ++i) {
        if (order) order[i] = prog.order[i];
        if (pass_of) pass_of[i] = prog.pass_of[i];
    }
    if (tile_mask)
        for (size_t p = 0; p < prog.passes.size(); ++p) {
            uint64_t m = 0;
            for (int j = 0; j < prog.passes[p].k; ++j) m |= uint64_t(1) << prog.passes[p].bits[j];
            tile_mask[p] = m;
        }
    *npasses = int64_t(prog.passes.size());
    return SV_OK;
}
