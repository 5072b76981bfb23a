// Dense k-qubit blocks: a 2^k x 2^k complex matrix M applied to k qubits.
//
// This is the definition X = I (x) ... (x) U (x) ... (x) I of sec. 2.2.1 with
// a 2^k block in place of the 2x2 U: for every basis index whose k block
// bits are 0 (a "group"), the 2^k amplitudes of the group are gathered,
// multiplied by M and scattered back.  Local block index i has qubits[0] as
// its most significant bit.
//
// complex64, k = 4 or 5: the group vectors are columns of a real matrix
// X (2^{k+1} x groups: real parts over imaginary parts) and the block is the
// real embedding A = [[Re M, -Im M], [Im M, Re M]], so Y = A X is a real
// GEMM run on FP32 MFMA (v_mfma_f32_32x32x2f32; 32-row blocks of A, steps of
// 2 along K).  A workgroup stages a tile of 4096 amplitudes (the k block bits
// plus the lowest other bits) in LDS; each wavefront owns 32-group column
// blocks: it reads its B operands from LDS, runs the MFMA chain with A held
// in registers, and writes the results back to the same LDS locations
// (columns are private to the wavefront, so no barrier is needed between
// reading and writing).  On MI355X FP32 MFMA runs at about 2.3x the FP32
// vector FMA rate available here (packed FP32 is not used).
// Other cases (complex128, whose FP64 MFMA rate equals the FP64 vector rate,
// or k < 4): one thread per group, the group in registers, M in LDS.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <vector>

#include "device_common.h"

using namespace svd;

namespace {

constexpr int kDTile = 12;  // log2 amplitudes per MFMA tile
constexpr int kDThreads = 256;
constexpr int kMaxK = 6;

struct DenseDesc {
    int8_t tile_bits[16];   // ascending global positions of the tile bits
    int8_t blk_local[8];    // local (tile) position of block bit j (j = 0: least significant bit of i)
    int8_t grp_local[16];   // local positions of the group bits, ascending
    int32_t ntile;
    int32_t nlow;           // tile_bits[0..nlow-1] == 0..nlow-1
};

template <int K>
__device__ __forceinline__ uint64_t dtile_index(uint64_t base, uint32_t r, uint32_t lowmask, int nlow,
                                                const int8_t *bits) {
    uint64_t g = base | (r & lowmask);
#pragma unroll
    for (int i = 0; i < K; ++i)
        if (i >= nlow) g |= uint64_t((r >> i) & 1) << bits[i];
    return g;
}

typedef float v16f __attribute__((ext_vector_type(16)));

// KB = k (4 or 5).  D = 2^k amplitudes per group, NRB = 2D/32 row blocks of
// A, D steps of K = 2.  Tile 2^12 amplitudes: 2^(12-k) groups, i.e. 2^(7-k)
// column blocks of 32 per wavefront over 4 wavefronts.
template <int KB>
__global__ __launch_bounds__(kDThreads) void k_dense_mfma(c64 *__restrict__ a, DenseDesc desc,
                                                          const float *__restrict__ aop, uint64_t nvb) {
    constexpr int D = 1 << KB;
    constexpr int NRB = (2 * D) / 32;
    constexpr int TILE = 1 << kDTile;
    constexpr int NGRP = TILE / D;
    constexpr int CPW = NGRP / 32 / (kDThreads / 64);  // column blocks per wavefront
    __shared__ c64 tile[TILE];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, h = lane >> 5;
    const uint32_t lowmask = (1u << desc.nlow) - 1;

    // A operand in registers: aop[(rb * D + s) * 64 + lane] = A[rb*32 + lane%32][2s + lane/32]
    float av[NRB][D];
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
        for (int s = 0; s < D; ++s) av[rb][s] = aop[(rb * D + s) * 64 + lane];

    // local offset of block index i
    uint32_t ioff[D];
#pragma unroll
    for (int i = 0; i < D; ++i) {
        uint32_t x = 0;
#pragma unroll
        for (int j = 0; j < KB; ++j)
            if ((i >> j) & 1) x |= 1u << desc.blk_local[j];
        ioff[i] = x;
    }

    // Workgroups walk tiles; the next tile's amplitudes are loaded into
    // registers while the current one multiplies.  Past the last tile the
    // load reads the current tile again (its values are not used), so that
    // no load is conditional.
    auto tile_base = [&](uint64_t t) {
#pragma unroll
        for (int i = 0; i < kDTile; ++i) t = insert_zero(t, desc.tile_bits[i]);
        return t;
    };
    c64 nv[TILE / kDThreads];
    auto load = [&](uint64_t b) {
#pragma unroll
        for (int j = 0; j < TILE / kDThreads; ++j)
            nv[j] = ldnt(a + dtile_index<kDTile>(b, uint32_t(tid + j * kDThreads), lowmask, desc.nlow, desc.tile_bits));
    };
    uint64_t nbase = tile_base(blockIdx.x);
    if (uint64_t(blockIdx.x) < nvb) load(nbase);
    for (uint64_t vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
        const uint64_t base = nbase;
#pragma unroll
        for (int j = 0; j < TILE / kDThreads; ++j) tile[tid + j * kDThreads] = nv[j];
        __syncthreads();
        if (vb + gridDim.x < nvb) nbase = tile_base(vb + gridDim.x);
        load(nbase);
#pragma unroll
        for (int cb = 0; cb < CPW; ++cb) {
            const uint32_t g = uint32_t((wave * CPW + cb) * 32 + (lane & 31));
            uint32_t gpart = 0;
#pragma unroll
            for (int j = 0; j < kDTile - KB; ++j)
                if ((g >> j) & 1) gpart |= 1u << desc.grp_local[j];
            // B operand of step s: X[2s + h][column] = part (2s+h)/D of amplitude (2s+h)%D
            float bv[D];
#pragma unroll
            for (int s = 0; s < D; ++s) {
                const int k0 = 2 * s, k1 = 2 * s + 1;
                const uint32_t r = gpart | (h ? ioff[k1 % D] : ioff[k0 % D]);
                const bool im = h ? (k1 >= D) : (k0 >= D);
                const c64 x = tile[r];
                bv[s] = im ? x.y : x.x;
            }
            v16f acc[NRB];
#pragma unroll
            for (int rb = 0; rb < NRB; ++rb) {
                acc[rb] = v16f{};
#pragma unroll
                for (int s = 0; s < D; ++s) acc[rb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[rb][s], bv[s], acc[rb], 0, 0, 0);
            }
            // D register v of lane: row 8(v/4) + 4h + v%4 of the row block
#pragma unroll
            for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int row0 = rb * 32 + 8 * (v / 4) + (v % 4);  // h = 0
                    const int row1 = row0 + 4;                         // h = 1
                    const uint32_t r = gpart | (h ? ioff[row1 % D] : ioff[row0 % D]);
                    const bool im = h ? (row1 >= D) : (row0 >= D);
                    float *dst = reinterpret_cast<float *>(&tile[r]) + (im ? 1 : 0);
                    *dst = acc[rb][v];
                }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < TILE / kDThreads; ++j) {
            const uint32_t r = uint32_t(tid + j * kDThreads);
            stnt(tile[r], a + dtile_index<kDTile>(base, r, lowmask, desc.nlow, desc.tile_bits));
        }
        __syncthreads();  // the next tile overwrites LDS
    }
}

// Direct form (block bits all >= 5): no LDS.  The operand layouts of
// v_mfma_f32_32x32x2f32 line up with the real embedding: for the 32 groups
// of a column block (consecutive group counters, so consecutive addresses),
// lane l = 32h + c of a wavefront feeds B rows 2s + h, i.e. the real and then
// the imaginary part of the amplitudes of parity h of group c, so it loads
// exactly those 2^KB/2 amplitudes; and the D registers of that lane hold the
// real and imaginary parts of whole output amplitudes of group c, which it
// stores back to where they came from.  Each wavefront walks column blocks
// with the A operand kept in registers.
struct DenseOff {
    uint64_t off[32];  // global offset of block index i
};

template <int KB>
__global__ __launch_bounds__(256) void k_dense_mfma_direct(c64 *__restrict__ a, BitSpec spec, DenseOff doff,
                                                           const float *__restrict__ aop, uint64_t ncb) {
    constexpr int D = 1 << KB;
    constexpr int NRB = (2 * D) / 32;
    constexpr int H = D / 2;  // amplitudes per lane
    const int lane = threadIdx.x & 63, h = lane >> 5, col = lane & 31;
    float av[NRB][D];
#pragma unroll
    for (int rb = 0; rb < NRB; ++rb)
#pragma unroll
        for (int st = 0; st < D; ++st) av[rb][st] = aop[(rb * D + st) * 64 + lane];
    // Offsets of disjoint block-index bits combine by OR: a lane's loads read
    // block index 2t + h (bit 0 is h) and its stores write row
    // 8 (v / 4) + 4 h + v % 4 (bit 2 is h), so each lane adds one offset of
    // its own to offsets common to the wavefront.
    const uint64_t hl = h ? doff.off[1] : 0, hs = h ? doff.off[4] : 0;
    // wavefront index (below 2^22) as a value the compiler knows is uniform,
    // so that the loop's branches and index arithmetic stay scalar
    const uint64_t wave = uint32_t(__builtin_amdgcn_readfirstlane(int((blockIdx.x * blockDim.x + threadIdx.x) >> 6)));
    const uint64_t nwaves = (uint64_t(gridDim.x) * blockDim.x) >> 6;
    if (wave >= ncb) return;
    // The group counter of lane col in column block cb is cb * 32 + col; its
    // bits are deposited around the block bits, and a deposit of disjoint
    // bits is the OR of their deposits: the lane's part is deposited once,
    // and the wavefront's part advances in deposited form, the carry
    // crossing the block bits through ((u | ~gm) + inc) & gm.  No index
    // work in the loop touches memory.
    const uint64_t gm = insert_zeros((ncb << 5) - 1, spec);
    const uint64_t inc = insert_zeros(nwaves << 5, spec);
    const uint64_t dcol = insert_zeros(uint64_t(col), spec);
    auto advance = [&](uint64_t u) { return ((u | ~gm) + inc) & gm; };
    // B rows 0..D-1 are real parts, D..2D-1 imaginary parts
    auto load = [&](float (&re)[H], float (&im)[H], uint64_t u) {
#pragma unroll
        for (int t = 0; t < H; ++t) {
            const c64 x = ldnt(a + (u | dcol | hl | doff.off[2 * t]));
            re[t] = x.x;
            im[t] = x.y;
        }
    };
    auto step = [&](const float (&re)[H], const float (&im)[H], uint64_t u) {
        const uint64_t base = u | dcol | hs;
        v16f acc[NRB];
#pragma unroll
        for (int rb = 0; rb < NRB; ++rb) acc[rb] = v16f{};
#pragma unroll
        for (int st = 0; st < D; ++st) {
            const float b = st < H ? re[st] : im[st - H];
#pragma unroll
            for (int rb = 0; rb < NRB; ++rb) acc[rb] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[rb][st], b, acc[rb], 0, 0, 0);
        }
        // D register v of the lane: row 32 rb + 8 (v / 4) + 4 h + v % 4
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const uint64_t off = base | doff.off[8 * (v / 4) + v % 4];
            if (NRB == 2) {
                // rows < 32 of row block 0 are real parts, row block 1 imaginary
                c64 o;
                o.x = acc[0][v];
                o.y = acc[NRB - 1][v];
                stnt(o, a + off);
            } else if (v < 8) {
                // one row block: rows < 16 real, rows >= 16 imaginary parts
                c64 o;
                o.x = acc[0][v];
                o.y = acc[0][v + 8];
                stnt(o, a + off);
            }
        }
    };
    // Two operand buffers, used in turn: the loads of a wavefront's next
    // column block are in flight while the MFMAs of the current one run.
    // Past the last block the prefetch reads the current block again (its
    // values are not used), so that no load is conditional.
    float xr[H], xi[H], yr[H], yi[H];
    uint64_t cb = wave, ux = insert_zeros(wave << 5, spec);
    load(xr, xi, ux);
    for (;;) {  // every branch is uniform over the wavefront
        const uint64_t c1 = cb + nwaves;
        const uint64_t uy = c1 < ncb ? advance(ux) : ux;
        load(yr, yi, uy);
        step(xr, xi, ux);
        if (c1 >= ncb) break;
        const uint64_t c2 = c1 + nwaves;
        const uint64_t un = c2 < ncb ? advance(uy) : uy;
        load(xr, xi, un);
        step(yr, yi, uy);
        if (c2 >= ncb) break;
        cb = c2;
        ux = un;
    }
}

// One thread per group: gather 2^KB amplitudes, multiply by M (in LDS),
// scatter.  goff[i] = global offset of block index i; group counter t has
// zero bits inserted at the block bit positions (ascending, in spec).
// NT: nontemporal loads and stores, for groups whose bases are (nearly)
// contiguous across lanes.  When the block holds the lowest index bits, lanes
// are 2^c amplitudes apart and each row load touches other lanes' lines; the
// cached form lets L2 serve the other rows.
template <typename T, int KB, bool NT>
__global__ __launch_bounds__(kDThreads) void k_dense_vec(T *__restrict__ a, uint64_t ngroups, BitSpec spec,
                                                         const typename RealOf<T>::type *__restrict__ mat,
                                                         const uint64_t *__restrict__ goff_g, uint64_t nvb) {
    using R = typename RealOf<T>::type;
    constexpr int D = 1 << KB;
    __shared__ R m[2 * D * D];
    __shared__ uint64_t goff[D];
    for (int i = threadIdx.x; i < 2 * D * D; i += kDThreads) m[i] = mat[i];
    for (int i = threadIdx.x; i < D; i += kDThreads) goff[i] = goff_g[i];
    __syncthreads();
    for (uint64_t vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
        const uint64_t t = vb * kDThreads + threadIdx.x;
        if (t >= ngroups) continue;
        const uint64_t base = insert_zeros(t, spec);
        T v[D];
#pragma unroll
        for (int i = 0; i < D; ++i) v[i] = NT ? ldnt(a + (base | goff[i])) : a[base | goff[i]];
        // rows stay a rolled loop (the group's inputs are already in
        // registers), two rows per trip: four independent accumulation
        // chains instead of two keep the FMA pipeline busy (measured at
        // n = 30, complex128, k = 5: 13.5 -> 9.6 ms; four rows per trip,
        // 12.0 ms)
#pragma unroll 1
        for (int r = 0; r < D; r += 2) {
            R re0 = 0, im0 = 0, re1 = 0, im1 = 0;
#pragma unroll
            for (int c = 0; c < D; ++c) {
                const R ar = m[2 * (r * D + c)], ai = m[2 * (r * D + c) + 1];
                const R br = m[2 * ((r + 1) * D + c)], bi = m[2 * ((r + 1) * D + c) + 1];
                re0 += ar * v[c].x - ai * v[c].y;
                im0 += ar * v[c].y + ai * v[c].x;
                re1 += br * v[c].x - bi * v[c].y;
                im1 += br * v[c].y + bi * v[c].x;
            }
            T o0, o1;
            o0.x = re0;
            o0.y = im0;
            o1.x = re1;
            o1.y = im1;
            if (NT) {
                stnt(o0, a + (base | goff[r]));
                stnt(o1, a + (base | goff[r + 1]));
            } else {
                a[base | goff[r]] = o0;
                a[base | goff[r + 1]] = o1;
            }
        }
    }
}

// Host preparation of one block: which kernel runs it, its launch
// descriptor and the operand bytes it reads from device memory.
struct DensePrep {
    int k = 0;
    bool mfma = false;
    bool direct = false;     // MFMA without LDS (block bits all >= 5)
    DenseOff doff{};         // direct: offsets of the block indices
    DenseDesc desc{};        // MFMA: tile layout
    BitSpec spec{};          // vector: zero bits of the group counter
    std::vector<char> bytes; // MFMA: A operand (float, lane order); vector: matrix then goff[]
};

// M is 2^k x 2^k complex, row-major, FP64, (re, im) interleaved; qs[0] is
// the most significant bit of the block index.
void dense_prepare(int n, int dtype, int k, const int *qs, const double *M, DensePrep &p) {
    const int D = 1 << k;
    int bpos[kMaxK];  // global bit of block index bit j (j = 0 least significant)
    for (int j = 0; j < k; ++j) bpos[j] = n - 1 - qs[k - 1 - j];
    uint64_t bmask = 0;
    for (int j = 0; j < k; ++j) bmask |= uint64_t(1) << bpos[j];
    p.k = k;
    p.mfma = dtype == SV_C64 && (k == 4 || k == 5) && n >= kDTile;
    bool low_free = true;
    for (int j = 0; j < k; ++j) low_free &= bpos[j] >= 5;
    p.direct = p.mfma && low_free && n >= k + 5;
    if (p.direct) {
        p.spec = svi_bits_of(bmask);
        for (int i = 0; i < D; ++i) {
            uint64_t x = 0;
            for (int j = 0; j < k; ++j)
                if ((i >> j) & 1) x |= uint64_t(1) << bpos[j];
            p.doff.off[i] = x;
        }
    }
    if (p.mfma) {
        DenseDesc &d = p.desc;
        std::memset(&d, 0, sizeof d);
        // tile = block bits + the lowest other bits, kDTile in all
        bool in_tile[64] = {false};
        for (int j = 0; j < k; ++j) in_tile[bpos[j]] = true;
        int cnt = k;
        for (int b = 0; b < n && cnt < kDTile; ++b)
            if (!in_tile[b]) {
                in_tile[b] = true;
                ++cnt;
            }
        int local[64];
        int nt = 0;
        for (int b = 0; b < n; ++b)
            if (in_tile[b]) {
                local[b] = nt;
                d.tile_bits[nt++] = int8_t(b);
            }
        d.ntile = nt;
        int nl = 0;
        while (nl < nt && d.tile_bits[nl] == nl) ++nl;
        d.nlow = nl;
        for (int j = 0; j < k; ++j) d.blk_local[j] = int8_t(local[bpos[j]]);
        int gi = 0;
        for (int i = 0; i < nt; ++i)
            if (!((bmask >> d.tile_bits[i]) & 1)) d.grp_local[gi++] = int8_t(i);
        // A operand in lane order: A = [[Re M, -Im M], [Im M, Re M]]
        const int nrb = (2 * D) / 32;
        p.bytes.resize(size_t(nrb) * D * 64 * sizeof(float));
        float *aop = reinterpret_cast<float *>(p.bytes.data());
        for (int rb = 0; rb < nrb; ++rb)
            for (int st = 0; st < D; ++st)
                for (int l = 0; l < 64; ++l) {
                    const int row = rb * 32 + (l & 31), col = 2 * st + (l >> 5);
                    const int ir = row % D, ic = col % D;
                    const double mr = M[2 * (ir * D + ic)], mi = M[2 * (ir * D + ic) + 1];
                    double val;
                    if (row < D)
                        val = col < D ? mr : -mi;
                    else
                        val = col < D ? mi : mr;
                    aop[size_t((rb * D + st) * 64 + l)] = float(val);
                }
        return;
    }
    const size_t rs = dtype == SV_C128 ? sizeof(double) : sizeof(float);
    p.bytes.resize(size_t(2) * D * D * rs + size_t(D) * sizeof(uint64_t));
    for (int i = 0; i < 2 * D * D; ++i) {
        if (dtype == SV_C128)
            reinterpret_cast<double *>(p.bytes.data())[i] = M[i];
        else
            reinterpret_cast<float *>(p.bytes.data())[i] = float(M[i]);
    }
    uint64_t *goff = reinterpret_cast<uint64_t *>(p.bytes.data() + size_t(2) * D * D * rs);
    for (int i = 0; i < D; ++i) {
        uint64_t x = 0;
        for (int j = 0; j < k; ++j)
            if ((i >> j) & 1) x |= uint64_t(1) << bpos[j];
        goff[i] = x;
    }
    p.spec = svi_bits_of(bmask);
}

// Launches a prepared block whose operand bytes are at dop (device).
hipError_t dense_launch(sv_state *s, const DensePrep &p, const void *dop) {
    const int n = s->n, k = p.k, D = 1 << k;
    if (p.direct) {
        // 2^(n-k-5) column blocks of 32 groups; each wavefront walks many of
        // them (its loads run one block ahead), so the grid is one workgroup
        // per compute unit by default, not one wavefront per block
        const uint64_t ncb = uint64_t(1) << (n - k - 5);
        const uint64_t nwg = (ncb + 3) / 4;
        const dim3 grid(unsigned(std::min<uint64_t>(nwg, uint64_t(svi_config().mfma_workgroups))));
        const float *aop = static_cast<const float *>(dop);
        if (k == 4)
            hipLaunchKernelGGL((k_dense_mfma_direct<4>), grid, dim3(256), 0, s->stream, static_cast<c64 *>(s->d),
                               p.spec, p.doff, aop, ncb);
        else
            hipLaunchKernelGGL((k_dense_mfma_direct<5>), grid, dim3(256), 0, s->stream, static_cast<c64 *>(s->d),
                               p.spec, p.doff, aop, ncb);
        return hipGetLastError();
    }
    if (p.mfma) {
        // workgroups walk tiles, two per compute unit by default: one
        // workgroup's LDS phases and barriers overlap the other's MFMAs
        // (n = 30: k = 4 at 3.25 ms with two, 3.5 ms with one; k = 5 at
        // 3.7 ms with two, 4.5 ms with one, 7.6 ms with a workgroup per tile)
        const uint64_t nvb = uint64_t(1) << (n - kDTile);
        const uint64_t wgs = 2 * uint64_t(svi_config().mfma_workgroups);
        const dim3 grid(unsigned(std::min<uint64_t>(nvb, wgs)));
        const float *aop = static_cast<const float *>(dop);
        if (k == 4)
            hipLaunchKernelGGL((k_dense_mfma<4>), grid, dim3(kDThreads), 0, s->stream, static_cast<c64 *>(s->d),
                               p.desc, aop, nvb);
        else
            hipLaunchKernelGGL((k_dense_mfma<5>), grid, dim3(kDThreads), 0, s->stream, static_cast<c64 *>(s->d),
                               p.desc, aop, nvb);
        return hipGetLastError();
    }
    const size_t rs = s->dtype == SV_C128 ? sizeof(double) : sizeof(float);
    const uint64_t ngroups = uint64_t(1) << (n - k);
    const uint64_t nvb = (ngroups + kDThreads - 1) / kDThreads;
    const dim3 grid(unsigned(std::min<uint64_t>(nvb, uint64_t(1) << 20)));
    const uint64_t *dgoff =
        reinterpret_cast<const uint64_t *>(static_cast<const char *>(dop) + size_t(2) * D * D * rs);
    int low_run = 0;  // block bits 0, 1, ... present
    while (low_run < p.spec.count && p.spec.pos[low_run] == low_run) ++low_run;
    const bool nt = low_run < 2;
#define SV_DVEC(T, KK)                                                                                               \
    do {                                                                                                             \
        if (nt)                                                                                                      \
            hipLaunchKernelGGL((k_dense_vec<T, KK, true>), grid, dim3(kDThreads), 0, s->stream, static_cast<T *>(s->d), \
                               ngroups, p.spec, static_cast<const typename RealOf<T>::type *>(dop), dgoff, nvb);     \
        else                                                                                                         \
            hipLaunchKernelGGL((k_dense_vec<T, KK, false>), grid, dim3(kDThreads), 0, s->stream,                     \
                               static_cast<T *>(s->d), ngroups, p.spec,                                             \
                               static_cast<const typename RealOf<T>::type *>(dop), dgoff, nvb);                     \
    } while (0)
    if (s->dtype == SV_C128) {
        switch (k) {
        case 1: SV_DVEC(c128, 1); break;
        case 2: SV_DVEC(c128, 2); break;
        case 3: SV_DVEC(c128, 3); break;
        case 4: SV_DVEC(c128, 4); break;
        case 5: SV_DVEC(c128, 5); break;
        default: SV_DVEC(c128, 6); break;
        }
    } else {
        switch (k) {
        case 1: SV_DVEC(c64, 1); break;
        case 2: SV_DVEC(c64, 2); break;
        case 3: SV_DVEC(c64, 3); break;
        case 4: SV_DVEC(c64, 4); break;
        case 5: SV_DVEC(c64, 5); break;
        default: SV_DVEC(c64, 6); break;
        }
    }
#undef SV_DVEC
    return hipGetLastError();
}

// Operand bytes of several blocks in one device buffer: offsets are 256-byte
// aligned; the buffer is freed in stream order after the last launch.
struct DenseUpload {
    void *dbuf = nullptr;
    std::vector<size_t> off;
};

hipError_t dense_upload(sv_state *s, const std::vector<DensePrep> &ps, DenseUpload &u) {
    size_t total = 0;
    u.off.resize(ps.size());
    for (size_t i = 0; i < ps.size(); ++i) {
        u.off[i] = total;
        total += (ps[i].bytes.size() + 255) & ~size_t(255);
    }
    if (total == 0) return hipSuccess;
    std::vector<char> host(total);
    for (size_t i = 0; i < ps.size(); ++i) std::memcpy(host.data() + u.off[i], ps[i].bytes.data(), ps[i].bytes.size());
    hipError_t e = hipMallocAsync(&u.dbuf, total, s->stream);
    if (e != hipSuccess) {
        u.dbuf = nullptr;
        return e;
    }
    e = hipMemcpyAsync(u.dbuf, host.data(), total, hipMemcpyHostToDevice, s->stream);
    // the host staging vector dies at return: wait for the copy to read it
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    return e;
}

}  // namespace

int svi_apply_dense(sv_state *s, int k, const int *qs, const double *M) {
    std::vector<DensePrep> ps(1);
    dense_prepare(s->n, s->dtype, k, qs, M, ps[0]);
    DenseUpload u;
    hipError_t e = dense_upload(s, ps, u);
    if (e == hipSuccess) e = dense_launch(s, ps[0], static_cast<char *>(u.dbuf) + u.off[0]);
    if (u.dbuf) (void)hipFreeAsync(u.dbuf, s->stream);
    return svi_fail(ps[0].mfma ? "sv_apply_fused (mfma)" : "sv_apply_fused (vector)", e);
}

extern "C" int sv_apply_fused(sv_state *s, int k, const int *qubits, const double *M) {
    if (!s || !qubits || !M || k < 1 || k > kMaxK || k > s->n) return SV_EINVAL;
    uint64_t seen = 0;
    for (int j = 0; j < k; ++j) {
        if (qubits[j] < 0 || qubits[j] >= s->n || ((seen >> qubits[j]) & 1)) return SV_EINVAL;
        seen |= uint64_t(1) << qubits[j];
    }
    const int D = 1 << k;
    for (int i = 0; i < 2 * D * D; ++i)
        if (!std::isfinite(M[i])) return SV_EINVAL;
    return svi_apply_dense(s, k, qubits, M);
}

// ------------------------------------------------------------------ block fusion
//
// Gates are clustered into dense blocks of at most kmax qubits (all qubits a
// gate touches: target, controls, both SWAP qubits).  The scan follows the
// same reordering rule as the fused-pass planner: a gate may move ahead of a
// deferred gate unless they share a qubit on which either acts
// non-diagonally.  Each block's matrix is composed on the host in FP64 and
// rounded once by the block kernel.  Gates on more than kmax qubits run as
// single gates.

namespace {

using cd = std::complex<double>;

struct BlockStep {
    bool single = false;
    int64_t gate = -1;     // single: source gate
    std::vector<int> qs;   // block: ascending qubit numbers (qs[0] = MSB of the block index)
    std::vector<cd> M;     // block: 2^k x 2^k row-major
    std::vector<int64_t> gates;  // source gates absorbed, in order
};

enum BMode : uint8_t { BM_NONE = 0, BM_DIAG = 1, BM_FULL = 2 };

// Qubits of a gate with their modes.
int gate_qubits(const PreparedGate &g, int n, int *q, uint8_t *mode) {
    int c = 0;
    if (g.kind == SV_G_SWAP) {
        q[c] = g.q;
        mode[c++] = BM_FULL;
        if (g.q2 != g.q) {
            q[c] = g.q2;
            mode[c++] = BM_FULL;
        }
        return c;
    }
    q[c] = g.q;
    mode[c++] = g.cls == GC_DIAG ? BM_DIAG : BM_FULL;
    for (uint64_t m = g.ctrl; m; m &= m - 1) {
        q[c] = n - 1 - __builtin_ctzll(m);
        mode[c++] = BM_DIAG;
    }
    return c;
}

// Full matrix of gate g on the ordered qubit list Q (Q[j] has local bit m-1-j).
void gate_on(const PreparedGate &g, int n, const std::vector<int> &Q, std::vector<cd> &G) {
    const int m = int(Q.size()), D = 1 << m;
    auto lbit = [&](int q) {
        for (int j = 0; j < m; ++j)
            if (Q[size_t(j)] == q) return m - 1 - j;
        return -1;
    };
    G.assign(size_t(D) * D, cd(0, 0));
    if (g.kind == SV_G_SWAP) {
        const int a = lbit(g.q), b = lbit(g.q2);
        for (int c = 0; c < D; ++c) {
            const int xa = (c >> a) & 1, xb = (c >> b) & 1;
            const int r = (c & ~((1 << a) | (1 << b))) | (xb << a) | (xa << b);
            G[size_t(r) * D + c] = 1.0;
        }
        return;
    }
    const int t = lbit(g.q);
    int cl = 0;
    for (uint64_t mm = g.ctrl; mm; mm &= mm - 1) cl |= 1 << lbit(n - 1 - __builtin_ctzll(mm));
    const cd u[2][2] = {{cd(g.U[0], g.U[1]), cd(g.U[2], g.U[3])}, {cd(g.U[4], g.U[5]), cd(g.U[6], g.U[7])}};
    for (int c = 0; c < D; ++c) {
        if ((c & cl) != cl) {
            G[size_t(c) * D + c] = 1.0;
            continue;
        }
        const int bit = (c >> t) & 1, c0 = c & ~(1 << t);
        G[size_t(c0) * D + c] += u[0][bit];
        G[size_t(c0 | (1 << t)) * D + c] += u[1][bit];
    }
}

// M over Q embedded in Q2 (Q a subset of Q2): identity on the new qubits.
void embed(const std::vector<cd> &M, const std::vector<int> &Q, const std::vector<int> &Q2, std::vector<cd> &out) {
    const int m = int(Q.size()), m2 = int(Q2.size()), D2 = 1 << m2;
    std::vector<int> pos(static_cast<size_t>(m));  // local bit in Q2 of Q[j]'s local bit
    int newmask = 0;
    for (int j2 = 0; j2 < m2; ++j2) newmask |= 1 << (m2 - 1 - j2);
    for (int j = 0; j < m; ++j)
        for (int j2 = 0; j2 < m2; ++j2)
            if (Q2[size_t(j2)] == Q[size_t(j)]) {
                pos[size_t(j)] = m2 - 1 - j2;
                newmask &= ~(1 << (m2 - 1 - j2));
            }
    auto extract = [&](int x) {
        int v = 0;
        for (int j = 0; j < m; ++j) v |= ((x >> pos[size_t(j)]) & 1) << (m - 1 - j);
        return v;
    };
    out.assign(size_t(D2) * D2, cd(0, 0));
    const int D = 1 << m;
    for (int r2 = 0; r2 < D2; ++r2)
        for (int c2 = 0; c2 < D2; ++c2) {
            if ((r2 & newmask) != (c2 & newmask)) continue;
            out[size_t(r2) * D2 + c2] = m ? M[size_t(extract(r2)) * D + extract(c2)] : M[0];
        }
}

void matmul(const std::vector<cd> &A, const std::vector<cd> &B, int D, std::vector<cd> &C) {
    C.assign(size_t(D) * D, cd(0, 0));
    for (int i = 0; i < D; ++i)
        for (int k = 0; k < D; ++k) {
            const cd a = A[size_t(i) * D + k];
            if (a == cd(0, 0)) continue;
            for (int j = 0; j < D; ++j) C[size_t(i) * D + j] += a * B[size_t(k) * D + j];
        }
}

std::vector<BlockStep> plan_blocks(int n, const PreparedGate *g, int64_t ng, int kmax) {
    std::vector<BlockStep> steps;
    std::vector<int64_t> rem(static_cast<size_t>(ng));
    for (int64_t i = 0; i < ng; ++i) rem[size_t(i)] = i;
    while (!rem.empty()) {
        int q0[64];
        uint8_t m0[64];
        const int c0 = gate_qubits(g[rem[0]], n, q0, m0);
        if (c0 > kmax) {
            BlockStep st;
            st.single = true;
            st.gate = rem[0];
            st.gates.push_back(rem[0]);
            steps.push_back(std::move(st));
            rem.erase(rem.begin());
            continue;
        }
        uint8_t blk[64] = {0};
        std::vector<int> Q;
        std::vector<cd> M(1, cd(1, 0)), tmp, G, M2;
        BlockStep st;
        std::vector<int64_t> deferred;
        size_t i = 0;
        for (; i < rem.size(); ++i) {
            const PreparedGate &x = g[rem[i]];
            int q[64];
            uint8_t md[64];
            const int c = gate_qubits(x, n, q, md);
            bool ok = true;
            for (int j = 0; j < c && ok; ++j)
                ok = !(blk[q[j]] == BM_FULL || (blk[q[j]] == BM_DIAG && md[j] == BM_FULL));
            std::vector<int> Q2 = Q;
            if (ok) {
                for (int j = 0; j < c; ++j)
                    if (std::find(Q2.begin(), Q2.end(), q[j]) == Q2.end()) Q2.push_back(q[j]);
                ok = int(Q2.size()) <= kmax;
            }
            if (ok) {
                std::sort(Q2.begin(), Q2.end());
                embed(M, Q, Q2, tmp);
                gate_on(x, n, Q2, G);
                matmul(G, tmp, 1 << int(Q2.size()), M2);
                M.swap(M2);
                Q.swap(Q2);
                st.gates.push_back(rem[i]);
            } else {
                deferred.push_back(rem[i]);
                for (int j = 0; j < c; ++j)
                    if (blk[q[j]] < md[j]) blk[q[j]] = md[j];
                bool all = true;
                for (int b = 0; b < n && all; ++b) all = blk[b] == BM_FULL;
                if (all) {
                    ++i;
                    break;
                }
            }
        }
        for (; i < rem.size(); ++i) deferred.push_back(rem[i]);
        st.qs = Q;
        st.M.swap(M);
        steps.push_back(std::move(st));
        rem.swap(deferred);
    }
    return steps;
}

int block_kmax() { return svi_config().block_qubits; }

}  // namespace

int svi_run_blocks(sv_state *s, const PreparedGate *gates, int64_t ng, bool prof) {
    const std::vector<BlockStep> steps = plan_blocks(s->n, gates, ng, block_kmax());
    // host preparation of every block, then one upload, then the launches
    std::vector<DensePrep> ps;
    std::vector<int> prep_of(steps.size(), -1);
    for (size_t i = 0; i < steps.size(); ++i) {
        const BlockStep &st = steps[i];
        if (st.single || st.qs.empty()) continue;
        std::vector<int> qs = st.qs;
        std::vector<cd> M = st.M;
        // complex64 blocks below 4 qubits: pad with identity qubits so the
        // block still runs on MFMA
        if (s->dtype == SV_C64 && s->n >= kDTile && qs.size() < 4) {
            std::vector<int> Q2 = qs;
            for (int q = s->n - 1; q >= 0 && Q2.size() < 4; --q)
                if (std::find(Q2.begin(), Q2.end(), q) == Q2.end()) Q2.push_back(q);
            std::sort(Q2.begin(), Q2.end());
            std::vector<cd> M2;
            embed(M, qs, Q2, M2);
            qs.swap(Q2);
            M.swap(M2);
        }
        prep_of[i] = int(ps.size());
        ps.emplace_back();
        dense_prepare(s->n, s->dtype, int(qs.size()), qs.data(), reinterpret_cast<const double *>(M.data()),
                      ps.back());
    }
    DenseUpload u;
    hipError_t e = dense_upload(s, ps, u);
    if (e != hipSuccess) {
        if (u.dbuf) (void)hipFreeAsync(u.dbuf, s->stream);
        return svi_fail("sv_run (block operands)", e);
    }
    int rc = SV_OK;
    for (size_t i = 0; i < steps.size() && rc == SV_OK; ++i) {
        const BlockStep &st = steps[i];
        if (st.single) {
            const PreparedGate &x = gates[st.gate];
            const int slot = svi_prof_begin(s, prof, x.kind == SV_G_SWAP ? STEP_SWAP : STEP_GATE);
            e = x.kind == SV_G_SWAP ? svi_launch_swap(s, x.q, x.q2) : svi_launch_gate(s, x.ctrl, x.q, x.U);
            svi_prof_end(s, slot);
            if (e != hipSuccess) rc = svi_fail("sv_run (single gate)", e);
            continue;
        }
        if (prep_of[i] < 0) continue;
        const int slot = svi_prof_begin(s, prof, STEP_BLOCK);
        e = dense_launch(s, ps[size_t(prep_of[i])], static_cast<char *>(u.dbuf) + u.off[size_t(prep_of[i])]);
        svi_prof_end(s, slot);
        if (e != hipSuccess) rc = svi_fail("sv_run (dense block)", e);
    }
    if (u.dbuf) (void)hipFreeAsync(u.dbuf, s->stream);
    return rc;
}

extern "C" int sv_plan_blocks(int n, const sv_gate *gates, int64_t ng, int kmax, int64_t *nsteps, int32_t *info,
                              double *mats, int64_t cap) {
    if (n < 1 || n > SV_MAX_QUBITS || ng < 0 || (ng > 0 && !gates) || !nsteps || kmax < 1 || kmax > kMaxK)
        return SV_EINVAL;
    std::vector<PreparedGate> prep;
    int rc = svi_prepare(n, gates, ng, prep, nullptr);
    if (rc != SV_OK) return rc;
    const std::vector<BlockStep> steps = plan_blocks(n, prep.data(), ng, kmax);
    *nsteps = int64_t(steps.size());
    const size_t msz = size_t(2) << (2 * kmax);
    for (int64_t i = 0; i < *nsteps && i < cap; ++i) {
        const BlockStep &st = steps[size_t(i)];
        int32_t *r = info + 8 * i;
        r[0] = st.single ? 1 : 0;
        r[1] = st.single ? int32_t(st.gate) : int32_t(st.qs.size());
        for (int j = 0; j < 6; ++j) r[2 + j] = (!st.single && j < int(st.qs.size())) ? st.qs[size_t(j)] : -1;
        if (mats && !st.single)
            for (size_t e = 0; e < st.M.size(); ++e) {
                mats[size_t(i) * msz + 2 * e] = st.M[e].real();
                mats[size_t(i) * msz + 2 * e + 1] = st.M[e].imag();
            }
    }
    return SV_OK;
}
