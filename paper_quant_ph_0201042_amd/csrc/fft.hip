// The QFT of sec. 2.3.2 as an in-place FFT (the route sec. 2.3.2 and Table 1
// compare with the circuit): passes over blocks of at most 8 index bits
// (12 for the last block of a range that starts at index bit 0), from the
// most significant bits of the transformed range down, each an HBM sweep.
//
// With x the sub-register index (bits [lo, lo + m)), qubit 0 its most
// significant bit, the circuit's gates on a block of qubits Q (H and the
// controlled R_k among them) form a t-qubit QFT without its swaps, and the
// controlled R_k whose target is in Q and whose control lies below the block
// commute with every later gate of the block.  So the block's pass is:
//   1. a DFT of size T = 2^t over the block bits v (sign s = +1 for the
//      QFT, -1 for its inverse), written in place at the bit-reversed
//      position u = rev_t(w) of each output w;
//   2. the phase of the lower controls, e^{2 pi i s w L / 2^b}, L the value
//      of the sub-register bits below the block and b the number of
//      sub-register bits from lo to the block's top;
//   3. the 2^{-t/2} of the block's H gates.
// After all blocks the register holds the QFT with the bits of the range
// reversed, exactly as the circuit leaves it before its final swaps.
//
// A workgroup stages a tile of 2^12 amplitudes in LDS: the block bits plus
// the lowest other bits (contiguous HBM runs).  The block DFT is a four-step
// split T = 2^A 2^B: a DFT over the high A block bits (16 registers per
// thread, radix-2 decimation in frequency), the twiddle e^{2 pi i s v0 w0/T},
// a DFT over the low B bits.  Decimation in frequency leaves output w at the
// bit-reversed register position, which is where step 1 wants it.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "device_common.h"

using namespace svd;

namespace {

constexpr int kFftThreads = 256;
constexpr int kTileBits = 12;
constexpr int kTile = 1 << kTileBits;
constexpr int kMaxBlock = 8;

struct QftPass {
    int32_t blo, t, A, B, lo, eb;  // block bits [blo, blo + t); ebits[eb] == blo
    int32_t btw, shift, h;         // phase exponent modulo 2^btw, scaled by 2^shift into the m-bit tables
    int8_t ebits[12];              // global bit of each tile bit (ascending)
    int8_t s1_reg[4], s1_thr[8];   // tile bits of stage 1's register / thread index bits
    int8_t s2_reg[4], s2_thr[8];   // the same for stage 2
    double scale;                  // 2^{-t/2}
};

// e^{2 pi i s j / 2^k}: tw256[j] (k = 8), tw_lo[j] (k = m), tw_hi[j] = e^{2 pi i s j 2^h / 2^m}
struct QftTables {
    const double2 *tw256, *lo, *hi;
};

template <typename T>
__device__ __forceinline__ uint32_t fswz(uint32_t e) {
    constexpr int SB = sizeof(T) == 16 ? 4 : 5;
    return e ^ (((e >> SB) ^ (e >> (2 * SB))) & ((1u << SB) - 1));
}

template <typename T>
__device__ __forceinline__ T cmulz(T x, double2 w) {
    using R = typename RealOf<T>::type;
    const R wr = R(w.x), wi = R(w.y);
    T r;
    r.x = x.x * wr - x.y * wi;
    r.y = x.x * wi + x.y * wr;
    return r;
}

__device__ __forceinline__ uint32_t rev_bits(uint32_t x, int nb) { return __brev(x) >> (32 - nb) & ((1u << nb) - 1); }

// rev_bits for compile-time arguments, nb >= 0
constexpr int rev_const(int x, int nb) {
    int y = 0;
    for (int i = 0; i < nb; ++i) y |= ((x >> i) & 1) << (nb - 1 - i);
    return y;
}

// DFT of size 2^D along the high D bits of the register index, for each
// value of its low 4 - D bits; output frequency f lands at position rev_D(f).
template <typename T, int D>
__device__ __forceinline__ void dft_regs(T (&v)[16], const double2 *tw) {
    constexpr int BB = 4 - D;
#pragma unroll
    for (int lsp = D - 1; lsp >= 0; --lsp) {
        const int sp = 1 << lsp;
#pragma unroll
        for (int i = 0; i < (1 << D); ++i) {
            if (i & sp) continue;
            const int j = i & (sp - 1);
#pragma unroll
            for (int b = 0; b < (1 << BB); ++b) {
                const int r0 = (i << BB) | b, r1 = ((i + sp) << BB) | b;
                const T x = v[r0], y = v[r1];
                T s, d;
                s.x = x.x + y.x;
                s.y = x.y + y.y;
                d.x = x.x - y.x;
                d.y = x.y - y.y;
                v[r0] = s;
                v[r1] = j == 0 ? d : cmulz(d, tw[j * (128 >> lsp)]);  // e^{2 pi i s j / (2 sp)}
            }
        }
    }
}

__device__ __forceinline__ uint32_t dep_bits(uint32_t x, const int8_t *pos, int nb) {
    uint32_t e = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i)
        if (i < nb) e |= ((x >> i) & 1u) << pos[i];
    return e;
}

__device__ __forceinline__ uint64_t dep_global(uint32_t e, const QftPass &P) {
    uint64_t g = 0;
#pragma unroll
    for (int i = 0; i < kTileBits; ++i) g |= uint64_t((e >> i) & 1u) << P.ebits[i];
    return g;
}

// Four-step twiddle after stage 1: e^{2 pi i s v0 w0 / T}.  It exists only
// when B > 0, hence t > 4 and A = 4: all 16 registers are the DFT dimension,
// v0 (the block's low bits) is fixed per thread, and register rev_4(w0)
// takes z0^w0 with z0 = e^{2 pi i s v0 / T}.
template <typename T>
__device__ __forceinline__ void four_step(T (&v)[16], const double2 *tw256, uint32_t v0, int t) {
    const double2 z0 = tw256[(v0 << (8 - t)) & 255];
    double2 p = z0;
#pragma unroll
    for (int w0 = 1; w0 < 16; ++w0) {
        const int r = int(__builtin_bitreverse32(uint32_t(w0)) >> 28);
        v[r] = cmulz(v[r], p);
        if (w0 < 15) {
            const double pr = p.x * z0.x - p.y * z0.y;
            p.y = p.x * z0.y + p.y * z0.x;
            p.x = pr;
        }
    }
}

// Phase of the lower controls and the scale, then the store: output
// w = rev_A(d1) + 2^A rev_B(d0) sits at block bits (d1, d0) of element e.
template <typename T>
__device__ __forceinline__ void finish_store(T *__restrict__ a, T x, uint32_t e, uint64_t g, const QftPass &P,
                                             const QftTables &tb) {
    const uint32_t amask = (1u << P.A) - 1, bmask = (1u << P.B) - 1;
    const uint32_t w = rev_bits((e >> (P.eb + P.B)) & amask, P.A) |
                       (P.B ? rev_bits((e >> P.eb) & bmask, P.B) << P.A : 0u);
    const uint64_t L = (g >> P.lo) & ((uint64_t(1) << (P.blo - P.lo)) - 1);
    const uint64_t k = ((uint64_t(w) * L) & ((uint64_t(1) << P.btw) - 1)) << P.shift;
    const double2 zl = tb.lo[k & ((uint64_t(1) << P.h) - 1)], zh = tb.hi[k >> P.h];
    double2 z;
    z.x = (zl.x * zh.x - zl.y * zh.y) * P.scale;
    z.y = (zl.x * zh.y + zl.y * zh.x) * P.scale;
    stnt(cmulz(x, z), a + g);
}

// One workgroup per tile of 2^12 amplitudes.  MODE 1 and 2, direct (block
// above the tile's 4 lowest bits): stage 1 loads its registers straight
// from HBM (its thread bits are the lowest tile bits outside the block's
// high part, so a wavefront reads runs of 2^4 or more amplitudes) and stage
// 2 stores straight to HBM; the tile crosses LDS once, between the stages
// (not at all when B = 0).  MODE 2 (a two-stage block at the top of the
// tile) computes the phases as powers of one value per thread, MODE 1 reads
// them from the tables per element.  MODE 0 (the block holds the lowest
// bits, which a stage keeps in registers): the tile is loaded and stored
// through LDS in contiguous runs and both stages work on it there.
template <typename T, int A, int B, int MODE>
__global__ __launch_bounds__(kFftThreads, 2) void k_qft_block(T *__restrict__ a, QftPass P, QftTables tb,
                                                              uint64_t ntiles) {
    constexpr bool DIRECT = MODE != 0;
    __shared__ T lds[(B > 0 || !DIRECT) ? kTile : 1];
    const uint32_t toff1 = dep_bits(threadIdx.x, P.s1_thr, 8);
    const uint32_t toff2 = B > 0 ? dep_bits(threadIdx.x, P.s2_thr, 8) : 0u;
    const uint64_t g1 = dep_global(toff1, P), g2 = dep_global(toff2, P);
    const uint64_t gtid = dep_global(threadIdx.x, P);  // tile bits 0..7
    {
        const uint64_t tile = blockIdx.x;  // one tile per workgroup (no loop keeps addresses out of registers)
        if (tile >= ntiles) return;
        uint64_t base = tile;
        for (int i = 0; i < kTileBits; ++i) base = insert_zero(base, P.ebits[i]);
        T v[16];
        if constexpr (DIRECT) {
#pragma unroll
            for (int r = 0; r < 16; ++r)
                v[r] = ldnt(a + (base | g1 | dep_global(dep_bits(uint32_t(r), P.s1_reg, 4), P)));
        } else {
#pragma unroll 4
            for (int r = 0; r < 16; ++r)
                lds[fswz<T>(uint32_t(r) * kFftThreads + threadIdx.x)] =
                    ldnt(a + (base | gtid | dep_global(uint32_t(r) << 8, P)));
            __syncthreads();
#pragma unroll
            for (int r = 0; r < 16; ++r) v[r] = lds[fswz<T>(toff1 | dep_bits(uint32_t(r), P.s1_reg, 4))];
        }
        dft_regs<T, A>(v, tb.tw256);
        if constexpr (B > 0) {
            four_step(v, tb.tw256, (toff1 >> P.eb) & ((1u << P.B) - 1), P.t);
#pragma unroll
            for (int r = 0; r < 16; ++r) lds[fswz<T>(toff1 | dep_bits(uint32_t(r), P.s1_reg, 4))] = v[r];
            __syncthreads();
#pragma unroll
            for (int r = 0; r < 16; ++r) v[r] = lds[fswz<T>(toff2 | dep_bits(uint32_t(r), P.s2_reg, 4))];
            dft_regs<T, B>(v, tb.tw256);
        }
        const uint32_t toff = B > 0 ? toff2 : toff1;
        const uint64_t gt = B > 0 ? g2 : g1;
        if constexpr (MODE == 2) {
            static_assert(A == 4 && B > 0, "powered phases need a two-stage block");
            // Block of 4 + B bits at the top of the tile, above its low
            // bits (MODE 2; every direct 8-bit block is there).  In
            // stage 2 the bits below the block are thread bits, so L is
            // fixed per thread and the phase is Z^w, Z = e^{2 pi i s L /
            // 2^btw}, with w = rev_4(d1) + 16 rev_B(d0): the low B bits
            // of d1 are thread bits (a fixed part wt of w), its top 4 - B
            // bits the low register bits (u = their reversal), d0 the
            // high register bits (v = rev_B(d0)).  Register (v, u) takes
            // scale Z^wt Z^{16 v} Z^u, built by repeated multiplication
            // from binary powers.
            constexpr int NU = 4 - B;
            const uint64_t L = ((base | gt) >> P.lo) & ((uint64_t(1) << (P.blo - P.lo)) - 1);
            const uint64_t k = (L & ((uint64_t(1) << P.btw) - 1)) << P.shift;
            const double2 zl = tb.lo[k & ((uint64_t(1) << P.h) - 1)], zh = tb.hi[k >> P.h];
            double2 Z;
            Z.x = zl.x * zh.x - zl.y * zh.y;
            Z.y = zl.x * zh.y + zl.y * zh.x;
            const uint32_t wt = rev_bits((toff >> (P.eb + B)) & ((1u << B) - 1), B) << NU;
            double2 c, q = Z;  // c = scale Z^wt by binary powering
            c.x = P.scale;
            c.y = 0.0;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if ((wt >> i) & 1u) {
                    const double cr = c.x * q.x - c.y * q.y;
                    c.y = c.x * q.y + c.y * q.x;
                    c.x = cr;
                }
                const double qr = q.x * q.x - q.y * q.y;
                q.y = 2.0 * q.x * q.y;
                q.x = qr;  // after the loop q = Z^16
            }
#pragma unroll
            for (int vv = 0; vv < (1 << B); ++vv) {
                double2 cu = c;
#pragma unroll
                for (int u = 0; u < (1 << NU); ++u) {
                    const int r = (rev_const(vv, B) << NU) | rev_const(u, NU);
                    const uint32_t re = dep_bits(uint32_t(r), P.s2_reg, 4);
                    stnt(cmulz(v[r], cu), a + (base | gt | dep_global(re, P)));
                    if (u + 1 < (1 << NU)) {
                        const double cr = cu.x * Z.x - cu.y * Z.y;
                        cu.y = cu.x * Z.y + cu.y * Z.x;
                        cu.x = cr;
                    }
                }
                const double cr = c.x * q.x - c.y * q.y;
                c.y = c.x * q.y + c.y * q.x;
                c.x = cr;
            }
        } else if constexpr (DIRECT) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const uint32_t re = dep_bits(uint32_t(r), B > 0 ? P.s2_reg : P.s1_reg, 4);
                finish_store(a, v[r], toff | re, base | gt | dep_global(re, P), P, tb);
            }
        } else {
            if constexpr (B > 0) __syncthreads();  // stage 2 has read the tile
#pragma unroll
            for (int r = 0; r < 16; ++r) lds[fswz<T>(toff | dep_bits(uint32_t(r), B > 0 ? P.s2_reg : P.s1_reg, 4))] = v[r];
            __syncthreads();
#pragma unroll 4
            for (int r = 0; r < 16; ++r) {
                const uint32_t e = uint32_t(r) * kFftThreads + threadIdx.x;
                finish_store(a, lds[fswz<T>(e)], e, base | gtid | dep_global(uint32_t(r) << 8, P), P, tb);
            }
        }
    }
}

// Register r of v takes z^{rev_4(r)}: v[rev_4(w)] *= z^w, w = 1..15.
template <typename T>
__device__ __forceinline__ void twiddle_powers(T (&v)[16], double2 z) {
    double2 p = z;
#pragma unroll
    for (int w = 1; w < 16; ++w) {
        const int r = int(__builtin_bitreverse32(uint32_t(w)) >> 28);
        v[r] = cmulz(v[r], p);
        if (w < 15) {
            const double pr = p.x * z.x - p.y * z.y;
            p.y = p.x * z.y + p.y * z.x;
            p.x = pr;
        }
    }
}

// A 12-bit block on the range's lowest bits, which start at index bit 0:
// the tile is the block.  DFT_4096 = DFT_16 (bits 8..11) x DFT_256, and
// DFT_256 = DFT_16 (bits 4..7) x DFT_16 (bits 0..3), each split with its
// twiddle; decimation in frequency puts w = w0 + 16 w1 + 256 w2 at
// rev_12(w).  No lower qubits: only the scale 2^-6 follows.  Stage 1 loads
// from HBM (64 consecutive amplitudes per wavefront), the tile crosses LDS
// between the stages and before the contiguous store.
template <typename T>
__global__ __launch_bounds__(kFftThreads, 2) void k_qft_block12(T *__restrict__ a, QftPass P, QftTables tb,
                                                                uint64_t ntiles) {
    __shared__ T lds[kTile];
    const uint32_t tid = threadIdx.x;
    // e^{2 pi i s tid / 4096} from the m-bit tables (m >= 12)
    const uint64_t kq = uint64_t(tid) << (P.shift + P.btw - 12);
    const double2 ql = tb.lo[kq & ((uint64_t(1) << P.h) - 1)], qh = tb.hi[kq >> P.h];
    double2 z1;
    z1.x = ql.x * qh.x - ql.y * qh.y;
    z1.y = ql.x * qh.y + ql.y * qh.x;
    const double2 z2 = tb.tw256[tid & 15u];  // e^{2 pi i s v_lo / 256}, v_lo = tid bits 0..3
    const uint32_t e2 = ((tid >> 4) << 8) | (tid & 15u);  // stage 2: thread -> bits 0..3, 8..11
    const uint32_t e3 = tid << 4;                        // stage 3: thread -> bits 4..11
    {
        const uint64_t tile = blockIdx.x;  // one tile per workgroup (no loop keeps addresses out of registers)
        if (tile >= ntiles) return;
        const uint64_t base = tile << kTileBits;
        T v[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = ldnt(a + (base | (uint64_t(r) << 8) | tid));
        dft_regs<T, 4>(v, tb.tw256);
        twiddle_powers(v, z1);
#pragma unroll
        for (int r = 0; r < 16; ++r) lds[fswz<T>((uint32_t(r) << 8) | tid)] = v[r];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = lds[fswz<T>(e2 | (uint32_t(r) << 4))];
        dft_regs<T, 4>(v, tb.tw256);
        twiddle_powers(v, z2);
#pragma unroll
        for (int r = 0; r < 16; ++r) lds[fswz<T>(e2 | (uint32_t(r) << 4))] = v[r];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = lds[fswz<T>(e3 | uint32_t(r))];
        dft_regs<T, 4>(v, tb.tw256);
        using R = typename RealOf<T>::type;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            v[r].x *= R(P.scale);
            v[r].y *= R(P.scale);
            lds[fswz<T>(e3 | uint32_t(r))] = v[r];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const uint32_t e = (uint32_t(r) << 8) | tid;
            stnt(lds[fswz<T>(e)], a + (base | e));
        }
    }
}

// ---------------------------------------------------------------- host

// Stage maps: the d tile bits of the DFT (ascending) on the high register
// bits, the highest 4 - d other tile bits on the low register bits, the
// remaining 8 (the lowest) on the thread index.
void stage_map(const std::vector<int> &dft, int8_t *reg, int8_t *thr) {
    std::vector<int> other;
    for (int b = 0; b < kTileBits; ++b) {
        bool in = false;
        for (int d : dft) in |= d == b;
        if (!in) other.push_back(b);
    }
    const int d = int(dft.size()), nb = 4 - d;
    for (int i = 0; i < 8; ++i) thr[i] = int8_t(other[size_t(i)]);
    for (int i = 0; i < nb; ++i) reg[i] = int8_t(other[size_t(8 + i)]);
    for (int i = 0; i < d; ++i) reg[nb + i] = int8_t(dft[size_t(i)]);
}

std::vector<QftPass> plan_qft(int n, int lo, int m) {
    std::vector<QftPass> out;
    const int h = (m + 1) / 2;
    // a range that starts at bit 0 ends with a 12-bit block whose tile is
    // itself (contiguous); the others take at most 8 bits, in as few blocks
    // as that allows, of balanced sizes: a smaller block leaves more of the
    // tile to the lowest bits, so longer contiguous runs (18 bits as 6 + 6 +
    // 6 rather than 8 + 8 + 2)
    const int last = (lo == 0 && m >= kTileBits) ? kTileBits : 0;
    for (int hi = lo + m; hi > lo;) {
        const int rest = hi - lo;  // bits of the range not yet transformed
        int t = last;
        if (rest != last) {
            const int upper = rest - last;
            const int nblk = (upper + kMaxBlock - 1) / kMaxBlock;
            t = (upper + nblk - 1) / nblk;
        }
        const int blo = hi - t;
        QftPass P;
        std::memset(&P, 0, sizeof P);
        P.blo = blo;
        P.t = t;
        P.A = std::min(4, t);
        P.B = t - P.A;
        P.lo = lo;
        P.btw = blo + t - lo;
        P.shift = m - P.btw;
        P.h = h;
        P.scale = std::ldexp(1.0, -(t / 2)) * ((t & 1) ? std::sqrt(0.5) : 1.0);
        const int c = kTileBits - t;
        std::vector<int> bits;
        if (blo >= c) {
            for (int b = 0; b < c; ++b) bits.push_back(b);
            for (int b = blo; b < blo + t; ++b) bits.push_back(b);
        } else {
            for (int b = 0; b < kTileBits; ++b) bits.push_back(b);
        }
        for (int i = 0; i < kTileBits; ++i) {
            P.ebits[i] = int8_t(bits[size_t(i)]);
            if (bits[size_t(i)] == blo) P.eb = i;
        }
        if (t <= kMaxBlock) {  // the 12-bit block's kernel has fixed maps
            std::vector<int> v1, v0;
            for (int i = 0; i < P.A; ++i) v1.push_back(P.eb + P.B + i);
            for (int i = 0; i < P.B; ++i) v0.push_back(P.eb + i);
            stage_map(v1, P.s1_reg, P.s1_thr);
            if (P.B > 0) stage_map(v0, P.s2_reg, P.s2_thr);
        }
        out.push_back(P);
        hi = blo;
    }
    return out;
}

struct TableKey {
    int device, m, sign;
    bool operator<(const TableKey &o) const { return std::tie(device, m, sign) < std::tie(o.device, o.m, o.sign); }
};

// Device twiddle tables per (device, m, sign), built once per process.
int tables_for(int device, int m, int sign, QftTables &out) {
    static std::mutex mu;
    static std::map<TableKey, QftTables> cache;
    std::lock_guard<std::mutex> lk(mu);
    const TableKey key{device, m, sign};
    auto it = cache.find(key);
    if (it != cache.end()) {
        out = it->second;
        return SV_OK;
    }
    const int h = (m + 1) / 2;
    const size_t nlo = size_t(1) << h, nhi = size_t(1) << (m - h);
    std::vector<double2> host(256 + nlo + nhi);
    const double two_pi = 6.283185307179586476925286766559;
    auto unit = [&](double frac) {  // e^{2 pi i s frac}, frac in [0, 1)
        double2 z;
        z.x = std::cos(two_pi * frac);
        z.y = sign * std::sin(two_pi * frac);
        return z;
    };
    for (int j = 0; j < 256; ++j) host[size_t(j)] = unit(j / 256.0);
    for (size_t j = 0; j < nlo; ++j) host[256 + j] = unit(std::ldexp(double(j), -m));
    for (size_t j = 0; j < nhi; ++j) host[256 + nlo + j] = unit(std::ldexp(double(j), h - m));
    void *d = nullptr;
    hipError_t e = hipMalloc(&d, host.size() * sizeof(double2));
    if (e != hipSuccess) return svi_fail("sv_qft: twiddle tables", e);
    e = hipMemcpy(d, host.data(), host.size() * sizeof(double2), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d);
        return svi_fail("sv_qft: twiddle upload", e);
    }
    QftTables t;
    t.tw256 = static_cast<const double2 *>(d);
    t.lo = t.tw256 + 256;
    t.hi = t.lo + nlo;
    cache[key] = t;
    out = t;
    return SV_OK;
}

template <typename T, int A, int B>
void launch_ab(sv_state *s, const QftPass &P, const QftTables &tb, dim3 grid, uint64_t ntiles) {
    // direct HBM stages unless the block holds one of the tile's 4 lowest
    // bits; powered phases for a two-stage block at the top of the tile
    T *a = static_cast<T *>(s->d);
    if constexpr (A == 4 && B > 0) {
        if (P.eb >= 4 && P.eb + P.t == kTileBits) {
            hipLaunchKernelGGL((k_qft_block<T, A, B, 2>), grid, dim3(kFftThreads), 0, s->stream, a, P, tb, ntiles);
            return;
        }
    }
    if (P.eb >= 4)
        hipLaunchKernelGGL((k_qft_block<T, A, B, 1>), grid, dim3(kFftThreads), 0, s->stream, a, P, tb, ntiles);
    else
        hipLaunchKernelGGL((k_qft_block<T, A, B, 0>), grid, dim3(kFftThreads), 0, s->stream, a, P, tb, ntiles);
}

// (A, B) is (t, 0) for t <= 4, else (4, t - 4).
template <typename T>
hipError_t launch_block(sv_state *s, const QftPass &P, const QftTables &tb, dim3 grid, uint64_t ntiles) {
    switch (P.A * 8 + P.B) {
    case 8: launch_ab<T, 1, 0>(s, P, tb, grid, ntiles); break;
    case 16: launch_ab<T, 2, 0>(s, P, tb, grid, ntiles); break;
    case 24: launch_ab<T, 3, 0>(s, P, tb, grid, ntiles); break;
    case 32: launch_ab<T, 4, 0>(s, P, tb, grid, ntiles); break;
    case 33: launch_ab<T, 4, 1>(s, P, tb, grid, ntiles); break;
    case 34: launch_ab<T, 4, 2>(s, P, tb, grid, ntiles); break;
    case 35: launch_ab<T, 4, 3>(s, P, tb, grid, ntiles); break;
    case 36: launch_ab<T, 4, 4>(s, P, tb, grid, ntiles); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

bool svi_qft_fft_ok(const sv_state *s) { return s->n >= kTileBits; }

int svi_qft_fft(sv_state *s, int lo, int m, int sign) {
    if (!svi_qft_fft_ok(s) || lo < 0 || m < 1 || lo + m > s->n) return SV_EINVAL;
    int device = s->device;
    if (device < 0 && hipGetDevice(&device) != hipSuccess) return SV_EDEVICE;
    QftTables tb;
    int rc = tables_for(device, m, sign, tb);
    if (rc != SV_OK) return rc;
    const uint64_t ntiles = uint64_t(1) << (s->n - kTileBits);  // at most 2^24 workgroups
    const dim3 grid(static_cast<unsigned>(ntiles));
    for (const QftPass &P : plan_qft(s->n, lo, m)) {
        hipError_t e;
        if (P.t == kTileBits) {
            if (s->dtype == SV_C128)
                hipLaunchKernelGGL((k_qft_block12<c128>), grid, dim3(kFftThreads), 0, s->stream,
                                   static_cast<c128 *>(s->d), P, tb, ntiles);
            else
                hipLaunchKernelGGL((k_qft_block12<c64>), grid, dim3(kFftThreads), 0, s->stream,
                                   static_cast<c64 *>(s->d), P, tb, ntiles);
            e = hipGetLastError();
        } else {
            e = s->dtype == SV_C128 ? launch_block<c128>(s, P, tb, grid, ntiles)
                                    : launch_block<c64>(s, P, tb, grid, ntiles);
        }
        if (e != hipSuccess) return svi_fail("sv_qft: block pass launch", e);
    }
    return SV_OK;
}

extern "C" int sv_qft_plan(int n, int q0, int m, int32_t *out, int64_t cap, int64_t *count) {
    if (!count || n < kTileBits || n > SV_MAX_QUBITS || q0 < 0 || m < 1 || q0 + m > n || cap < 0 ||
        (cap > 0 && !out))
        return SV_EINVAL;
    const std::vector<QftPass> plan = plan_qft(n, n - q0 - m, m);
    *count = int64_t(plan.size());
    for (size_t p = 0; p < plan.size() && int64_t(p) < cap; ++p) {
        const QftPass &P = plan[p];
        int32_t *o = out + p * SV_QFT_PLAN_WORDS;
        const int32_t head[6] = {P.blo, P.t, P.A, P.B, P.lo, P.eb};
        for (int i = 0; i < 6; ++i) o[i] = head[i];
        for (int i = 0; i < 12; ++i) o[6 + i] = P.ebits[i];
        const bool maps = P.t <= kMaxBlock;
        for (int i = 0; i < 4; ++i) o[18 + i] = maps ? P.s1_reg[i] : -1;
        for (int i = 0; i < 8; ++i) o[22 + i] = maps ? P.s1_thr[i] : -1;
        for (int i = 0; i < 4; ++i) o[30 + i] = maps && P.B ? P.s2_reg[i] : -1;
        for (int i = 0; i < 8; ++i) o[34 + i] = maps && P.B ? P.s2_thr[i] : -1;
    }
    return SV_OK;
}
