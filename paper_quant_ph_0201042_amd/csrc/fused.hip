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
#include <algorithm>
#include <cstring>
#include <vector>

#include "device_common.h"

using namespace svd;

SviConfig &svi_config() {
    static SviConfig c = {12, 13, 6, 512};
    return c;
}

namespace {

enum OpKind : int32_t { OP_DENSE = 0, OP_PERM = 1, OP_DIAG = 2 };

struct FOp {
    int32_t kind;
    int32_t lbit;    // local position of the target bit, -1 if outside the tile (diagonal only)
    uint32_t lctrl;  // controls inside the tile, as local bit positions
    int32_t last;    // 1 for the last op of the pass
    uint64_t gctrl;  // controls outside the tile, as global bits
    uint64_t gtbit;  // global target bit of a diagonal op outside the tile, else 0
    double m[8];
};
static_assert(sizeof(FOp) == 96, "FOp layout");

constexpr int kMaxTileBits = 16;
struct FPass {
    int32_t k;      // tile bits
    int32_t nlow;   // bits[0..nlow-1] == 0..nlow-1
    int32_t first;  // first op index
    int32_t nops;
    int8_t bits[kMaxTileBits];  // ascending global bit positions of the tile
};

template <int K>
__device__ __forceinline__ uint64_t tile_index(uint64_t base, uint32_t r, uint32_t lowmask, int nlow,
                                               const int8_t *bits) {
    uint64_t g = base | (r & lowmask);
#pragma unroll
    for (int i = 0; i < K; ++i)
        if (i >= nlow) g |= uint64_t((r >> i) & 1) << bits[i];
    return g;
}

template <typename T, int K, int NT>
__global__ __launch_bounds__(NT) void k_fused(T *__restrict__ a, const FPass *__restrict__ pass,
                                              const FOp *__restrict__ ops) {
    using R = typename RealOf<T>::type;
    constexpr uint32_t TILE = 1u << K;
    __shared__ T tile[TILE];
    const FPass P = *pass;
    const int tid = threadIdx.x;
    const uint32_t lowmask = (1u << P.nlow) - 1;
    uint64_t base = blockIdx.x;
#pragma unroll
    for (int i = 0; i < K; ++i) base = insert_zero(base, P.bits[i]);

    // load: thread tid takes local indices tid, tid + NT, ... (tiles smaller
    // than the workgroup leave the upper threads idle)
    constexpr int PER = TILE >= uint32_t(NT) ? int(TILE / NT) : 1;
    {
        T v[PER];
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const uint32_t r = uint32_t(tid + j * NT);
            if (r < TILE) v[j] = ldnt(a + tile_index<K>(base, r, lowmask, P.nlow, P.bits));
        }
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const uint32_t r = uint32_t(tid + j * NT);
            if (r < TILE) tile[r] = v[j];
        }
    }
    __syncthreads();

    const FOp *op = ops + P.first;
    for (int o = 0; o < P.nops; ++o, ++op) {
        const int kind = op->kind;
        const uint64_t gctrl = op->gctrl;
        const bool on = (base & gctrl) == gctrl;  // uniform over the workgroup
        const uint32_t lctrl = op->lctrl;
        if (on) {
            R m[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) m[i] = R(op->m[i]);
            if (kind == OP_DIAG) {
                const int lb = op->lbit;
                if (lb >= 0) {
#pragma unroll 4
                    for (uint32_t r = tid; r < TILE; r += NT) {
                        if ((r & lctrl) != lctrl) continue;
                        const int hi = (r >> lb) & 1;
                        tile[r] = hi ? cscale<T, R>(m[6], m[7], tile[r]) : cscale<T, R>(m[0], m[1], tile[r]);
                    }
                } else {
                    const bool hi = (base & op->gtbit) != 0;
                    const R fr = hi ? m[6] : m[0], fi = hi ? m[7] : m[1];
                    if (!(fr == R(1) && fi == R(0))) {
#pragma unroll 4
                        for (uint32_t r = tid; r < TILE; r += NT) {
                            if ((r & lctrl) != lctrl) continue;
                            tile[r] = cscale<T, R>(fr, fi, tile[r]);
                        }
                    }
                }
            } else {
                const int lb = op->lbit;
                const uint32_t tb = 1u << lb;
#pragma unroll 4
                for (uint32_t p = tid; p < TILE / 2; p += NT) {
                    const uint32_t r0 = uint32_t(insert_zero(p, lb));
                    if ((r0 & lctrl) != lctrl) continue;
                    const T x = tile[r0], y = tile[r0 | tb];
                    if (kind == OP_PERM) {
                        tile[r0] = y;
                        tile[r0 | tb] = x;
                    } else {
                        tile[r0] = mac2<T, R>(m, 0, x, y);
                        tile[r0 | tb] = mac2<T, R>(m, 4, x, y);
                    }
                }
            }
        }
        // elementwise ops keep the load mapping, so a run of diagonal ops
        // needs no barrier between them
        const bool next_diag = !op->last && op[1].kind == OP_DIAG;
        if (!(kind == OP_DIAG && next_diag)) __syncthreads();
    }
    if (P.nops == 0) __syncthreads();

#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const uint32_t r = uint32_t(tid + j * NT);
        if (r < TILE) stnt(tile[r], a + tile_index<K>(base, r, lowmask, P.nlow, P.bits));
    }
}

// ------------------------------------------------------------------ planner

enum Mode : uint8_t { M_NONE = 0, M_DIAG = 1, M_FULL = 2 };

struct PlannedPass {
    std::vector<int> bits;  // ascending tile bits
    int nlow;
    std::vector<FOp> ops;
    std::vector<int64_t> gate_ids;  // source gate of each op
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

std::vector<Step> plan(int n, const PreparedGate *g, int64_t ng, int K, int nlow_req, int max_ops) {
    std::vector<Step> steps;
    K = std::min(K, n);
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
        bool in_tile[64] = {false};
        for (int b = 0; b < nlow; ++b) in_tile[b] = true;
        int free_slots = K - nlow;
        uint8_t blk[64] = {0};
        std::vector<int64_t> sched, deferred;
        size_t i = head;
        for (; i < rem.size(); ++i) {
            const PreparedGate &x = g[rem[i]];
            if (x.kind == SV_G_SWAP) {
                // a permutation of two qubits: everything after it on those
                // qubits waits; other gates may still join this pass
                const int b1 = n - 1 - x.q, b2 = n - 1 - x.q2;
                deferred.push_back(rem[i]);
                block(blk, b1, M_FULL);
                block(blk, b2, M_FULL);
                continue;
            }
            const int tb = n - 1 - x.q;
            const bool diag = x.cls == GC_DIAG;
            const Mode tm = diag ? M_DIAG : M_FULL;
            bool ok = !conflicts(blk, tb, tm);
            for (uint64_t c = x.ctrl; ok && c; c &= c - 1) ok = !conflicts(blk, __builtin_ctzll(c), M_DIAG);
            if (ok && int(sched.size()) >= max_ops) ok = false;
            if (ok && !diag && !in_tile[tb]) {
                if (free_slots > 0) {
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
                block(blk, tb, tm);
                for (uint64_t c = x.ctrl; c; c &= c - 1) block(blk, __builtin_ctzll(c), M_DIAG);
                // stop scanning once every qubit is fully blocked
                bool all = true;
                for (int b = 0; b < n && all; ++b) all = blk[b] == M_FULL;
                if (all) {
                    ++i;
                    break;
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
        int local[64];
        for (int b = 0; b < n; ++b)
            if (in_tile[b]) {
                local[b] = int(p.bits.size());
                p.bits.push_back(b);
            }
        int nl = 0;
        while (nl < int(p.bits.size()) && p.bits[size_t(nl)] == nl) ++nl;
        p.nlow = nl;
        for (int64_t idx : sched) {
            const PreparedGate &x = g[idx];
            FOp op;
            std::memset(&op, 0, sizeof op);
            const int tb = n - 1 - x.q;
            op.kind = x.cls == GC_DIAG ? OP_DIAG : (x.cls == GC_PERM ? OP_PERM : OP_DENSE);
            op.lbit = in_tile[tb] ? local[tb] : -1;
            op.gtbit = in_tile[tb] ? 0 : (uint64_t(1) << tb);
            for (uint64_t c = x.ctrl; c; c &= c - 1) {
                const int cb = __builtin_ctzll(c);
                if (in_tile[cb])
                    op.lctrl |= 1u << local[cb];
                else
                    op.gctrl |= uint64_t(1) << cb;
            }
            for (int j = 0; j < 8; ++j) op.m[j] = x.U[j];
            p.ops.push_back(op);
            p.gate_ids.push_back(idx);
        }
        if (!p.ops.empty()) p.ops.back().last = 1;
        steps.push_back(std::move(st));
        rem.erase(rem.begin() + std::ptrdiff_t(head), rem.end());
        rem.insert(rem.end(), deferred.begin(), deferred.end());
    }
    return steps;
}

template <typename T, int K>
hipError_t launch_pass(sv_state *s, const FPass *dpass, const FOp *dops) {
    const uint64_t tiles = uint64_t(1) << (s->n - K);
    hipLaunchKernelGGL((k_fused<T, K, 256>), dim3(tiles), dim3(256), 0, s->stream, static_cast<T *>(s->d), dpass,
                       dops);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pass_k(sv_state *s, int K, const FPass *dpass, const FOp *dops) {
    switch (K) {
    case 1: return launch_pass<T, 1>(s, dpass, dops);
    case 2: return launch_pass<T, 2>(s, dpass, dops);
    case 3: return launch_pass<T, 3>(s, dpass, dops);
    case 4: return launch_pass<T, 4>(s, dpass, dops);
    case 5: return launch_pass<T, 5>(s, dpass, dops);
    case 6: return launch_pass<T, 6>(s, dpass, dops);
    case 7: return launch_pass<T, 7>(s, dpass, dops);
    case 8: return launch_pass<T, 8>(s, dpass, dops);
    case 9: return launch_pass<T, 9>(s, dpass, dops);
    case 10: return launch_pass<T, 10>(s, dpass, dops);
    case 11: return launch_pass<T, 11>(s, dpass, dops);
    case 12: return launch_pass<T, 12>(s, dpass, dops);
    case 13:
        if (sizeof(T) == 8) return launch_pass<T, 13>(s, dpass, dops);
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

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

int svi_run_fused(sv_state *s, const PreparedGate *gates, int64_t ng, bool prof) {
    const SviConfig &cfg = svi_config();
    const int K = s->dtype == SV_C128 ? cfg.fused_tile_bits_c128 : cfg.fused_tile_bits_c64;
    std::vector<Step> steps = plan(s->n, gates, ng, K, cfg.fused_low_bits, cfg.fused_max_ops);

    // pack descriptors: FPass array, then FOp array
    size_t npass = 0, nops = 0;
    for (const Step &st : steps)
        if (!st.is_swap) {
            ++npass;
            nops += st.pass.ops.size();
        }
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
    FPass *hp = static_cast<FPass *>(f->host);
    FOp *ho = reinterpret_cast<FOp *>(static_cast<char *>(f->host) + pass_bytes);
    size_t pi = 0, oi = 0;
    for (const Step &st : steps) {
        if (st.is_swap) continue;
        FPass P;
        std::memset(&P, 0, sizeof P);
        P.k = int32_t(st.pass.bits.size());
        P.nlow = st.pass.nlow;
        P.first = int32_t(oi);
        P.nops = int32_t(st.pass.ops.size());
        for (size_t j = 0; j < st.pass.bits.size(); ++j) P.bits[j] = int8_t(st.pass.bits[j]);
        hp[pi++] = P;
        for (const FOp &op : st.pass.ops) ho[oi++] = op;
    }
    if (hipMemcpyAsync(f->dev, f->host, bytes - 256, hipMemcpyHostToDevice, s->stream) != hipSuccess)
        return SV_EDEVICE;
    if (hipEventRecord(f->uploaded, s->stream) != hipSuccess) return SV_EDEVICE;

    const FPass *dp = static_cast<const FPass *>(f->dev);
    const FOp *dops = reinterpret_cast<const FOp *>(static_cast<char *>(f->dev) + pass_bytes);
    pi = 0;
    for (const Step &st : steps) {
        hipError_t e;
        const int slot = svi_prof_begin(s, prof, st.is_swap ? STEP_SWAP : STEP_FUSED_PASS);
        if (st.is_swap) {
            e = svi_launch_swap(s, st.q1, st.q2);
        } else {
            const int k = int(st.pass.bits.size());
            e = s->dtype == SV_C128 ? launch_pass_k<c128>(s, k, dp + pi, dops)
                                    : launch_pass_k<c64>(s, k, dp + pi, dops);
            ++pi;
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
    const SviConfig &cfg = svi_config();
    const int K = dtype == SV_C128 ? cfg.fused_tile_bits_c128 : cfg.fused_tile_bits_c64;
    const std::vector<Step> steps = plan(n, prep.data(), ng, K, cfg.fused_low_bits, cfg.fused_max_ops);
    int64_t pos = 0, pi = 0;
    for (const Step &st : steps) {
        for (int64_t id : st.pass.gate_ids) {
            if (order) order[pos] = id;
            if (pass_of) pass_of[pos] = st.is_swap ? -1 : int32_t(pi);
            ++pos;
        }
        if (!st.is_swap) {
            if (tile_mask) {
                uint64_t m = 0;
                for (int b : st.pass.bits) m |= uint64_t(1) << b;
                tile_mask[pi] = m;
            }
            ++pi;
        }
    }
    *npasses = pi;
    return pos == ng ? SV_OK : SV_EDEVICE;
}
