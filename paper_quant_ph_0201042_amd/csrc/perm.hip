// Permutation of index bits in one HBM pass: a run of SWAP gates whose
// product is an involution on the index bits (the ⌊n/2⌋ swaps that end the
// QFT of sec. 2.3.2 reverse the bit order) moves every amplitude once
// instead of once per swap.
//
// With f the bit map (bit b of j goes to bit f(b)) and f(f(b)) = b, the new
// register is new[j] = old[F(j)], F applying f to the bits of j.  The tile
// bits T are the lowest bits L and their images f(L); f maps T onto itself
// and the other ("middle") bits onto themselves, so the tile with middle
// value m exchanges its amplitudes with the tile of middle value F(m).  A
// workgroup loads both tiles into LDS (contiguous runs of 2^|L| amplitudes),
// then writes each tile from the other with the local bits permuted, again
// in contiguous runs.  Workgroups whose partner tile has a smaller middle
// value leave the pair to that partner.
//
// The workgroup index is spread over the middle bits in the order of
// max(b, f(b)), smallest first: workgroups that run at the same time then
// differ in bits that are low on both sides of the exchange, so both tiles
// of every pair in flight fall in a few memory pages.  For a bit reversal
// these are the bits nearest the middle of the index; taking the middle
// bits in ascending order instead spreads the F(m) side over thousands of
// pages: the n = 28 bit reversal took 4.27 ms that way, 3.28 ms this way.
#include <algorithm>

#include "device_common.h"

using namespace svd;

namespace {

constexpr int kPermThreads = 256;
// tiles of up to 2^10 amplitudes (runs of 2^5) exchange through two LDS
// tiles (32 KiB of complex128); tiles of up to 2^12 (runs of 2^6) through
// one LDS tile and registers (64 KiB)

struct BitPerm {
    int t;                   // tile bits
    int nm;                  // middle bits
    int8_t tbits[16];        // ascending global positions of the tile bits
    int8_t gloc[16];         // local bit i -> local bit of f(tbits[i])
    int8_t fmap[64];         // f on global bits
    int8_t mbits[64];        // bit j of the pair index -> global middle bit
};

template <int MT>
__device__ __forceinline__ uint64_t deposit_tile(uint32_t r, const BitPerm &P) {
    uint64_t g = 0;
#pragma unroll
    for (int i = 0; i < MT; ++i)
        if (i < P.t) g |= uint64_t((r >> i) & 1) << P.tbits[i];
    return g;
}

template <int MT>
__device__ __forceinline__ uint32_t permute_local(uint32_t r, const BitPerm &P) {
    uint32_t x = 0;
#pragma unroll
    for (int i = 0; i < MT; ++i)
        if (i < P.t) x |= ((r >> i) & 1u) << P.gloc[i];
    return x;
}

// LDS index with the bits above each bank window folded onto the
// bank-selecting low bits: the permuted reads of a bit reversal would
// otherwise put a whole wavefront on one bank.
template <typename T>
__device__ __forceinline__ uint32_t pswz(uint32_t r) {
    constexpr int SB = sizeof(T) == 16 ? 4 : 5;
    return r ^ (((r >> SB) ^ (r >> (2 * SB))) & ((1u << SB) - 1));
}

template <typename T, int MT>
__global__ __launch_bounds__(kPermThreads) void k_bitperm(T *__restrict__ a, BitPerm P, uint64_t nvb) {
    __shared__ T lds[2 << MT];
    const uint32_t tile = 1u << P.t;
    for (uint64_t vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
        uint64_t m = 0;
        for (int j = 0; j < P.nm; ++j) m |= ((vb >> j) & uint64_t(1)) << P.mbits[j];
        uint64_t mp = 0;  // F(m)
        for (uint64_t x = m; x; x &= x - 1) mp |= uint64_t(1) << P.fmap[__builtin_ctzll(x)];
        if (mp < m) continue;  // uniform over the workgroup
        const bool self = mp == m;
        __syncthreads();  // the previous pair's LDS reads are done
        for (uint32_t r = threadIdx.x; r < tile; r += kPermThreads) {
            const uint64_t d = deposit_tile<MT>(r, P);
            lds[pswz<T>(r)] = ldnt(a + (m | d));
            if (!self) lds[tile + pswz<T>(r)] = ldnt(a + (mp | d));
        }
        __syncthreads();
        // new[m | d(r)] = old[F(m) | d(g(r))], and the same with m, F(m) exchanged
        for (uint32_t r = threadIdx.x; r < tile; r += kPermThreads) {
            const uint64_t d = deposit_tile<MT>(r, P);
            const uint32_t src = permute_local<MT>(r, P);
            stnt(lds[(self ? 0u : tile) + pswz<T>(src)], a + (m | d));
            if (!self) stnt(lds[pswz<T>(src)], a + (mp | d));
        }
    }
}

// The same exchange with one tile of each pair in LDS and the other in
// registers (2^MT / 256 amplitudes per thread): half the LDS of the kernel
// above for the same tile, so tiles of 2^12 amplitudes (runs of 2^6
// contiguous amplitudes, 1 KiB of complex128) leave room for two
// workgroups per compute unit.  Per pair: tile m into LDS and tile F(m)
// into registers; F(m)'s places are written from LDS (tile m permuted);
// then the registers go through LDS and m's places are written.
template <typename T, int MT>
__global__ __launch_bounds__(kPermThreads) void k_bitperm_rl(T *__restrict__ a, BitPerm P, uint64_t nvb) {
    constexpr int R = (1 << MT) / kPermThreads;
    __shared__ T lds[1 << MT];
    const uint32_t tile = 1u << P.t;
    for (uint64_t vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
        uint64_t m = 0;
        for (int j = 0; j < P.nm; ++j) m |= ((vb >> j) & uint64_t(1)) << P.mbits[j];
        uint64_t mp = 0;  // F(m)
        for (uint64_t x = m; x; x &= x - 1) mp |= uint64_t(1) << P.fmap[__builtin_ctzll(x)];
        if (mp < m) continue;  // uniform over the workgroup
        const bool self = mp == m;
        __syncthreads();  // the previous pair's LDS reads are done
        T v[R];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const uint32_t r = threadIdx.x + uint32_t(k) * kPermThreads;
            if (r < tile) {
                const uint64_t d = deposit_tile<MT>(r, P);
                lds[pswz<T>(r)] = ldnt(a + (m | d));
                if (!self) v[k] = ldnt(a + (mp | d));
            }
        }
        __syncthreads();
        // new[F(m) | d(r)] = old[m | d(g(r))] (or new[m | d(r)] for a self pair)
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const uint32_t r = threadIdx.x + uint32_t(k) * kPermThreads;
            if (r < tile) stnt(lds[pswz<T>(permute_local<MT>(r, P))], a + (mp | deposit_tile<MT>(r, P)));
        }
        if (self) continue;
        __syncthreads();  // tile m's reads from LDS are done
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const uint32_t r = threadIdx.x + uint32_t(k) * kPermThreads;
            if (r < tile) lds[pswz<T>(r)] = v[k];
        }
        __syncthreads();
        // new[m | d(r)] = old[F(m) | d(g(r))]
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const uint32_t r = threadIdx.x + uint32_t(k) * kPermThreads;
            if (r < tile) stnt(lds[pswz<T>(permute_local<MT>(r, P))], a + (m | deposit_tile<MT>(r, P)));
        }
    }
}

}  // namespace

// f: bit map over the n index bits (an involution); returns
// hipErrorInvalidValue if it is not one.
hipError_t svi_launch_bitperm(sv_state *s, const int *f) {
    const int n = s->n;
    for (int b = 0; b < n; ++b)
        if (f[b] < 0 || f[b] >= n || f[f[b]] != b) return hipErrorInvalidValue;
    BitPerm P{};
    bool in_t[64] = {false};
    const int l = std::min(s->dtype == SV_C128 ? svi_config().perm_low_bits : svi_config().perm_low_bits_c64, n);
    for (int b = 0; b < l; ++b) {
        in_t[b] = true;
        in_t[f[b]] = true;
    }
    int t = 0;
    int loc[64];
    for (int b = 0; b < n; ++b)
        if (in_t[b]) {
            loc[b] = t;
            P.tbits[t++] = int8_t(b);
        }
    P.t = t;
    for (int i = 0; i < t; ++i) P.gloc[i] = int8_t(loc[f[P.tbits[i]]]);
    for (int b = 0; b < 64; ++b) P.fmap[b] = int8_t(b < n ? f[b] : b);
    int mid[64];
    int nm = 0;
    for (int b = 0; b < n; ++b)
        if (!in_t[b]) mid[nm++] = b;
    std::stable_sort(mid, mid + nm, [&](int x, int y) { return std::max(x, f[x]) < std::max(y, f[y]); });
    P.nm = nm;
    for (int j = 0; j < nm; ++j) P.mbits[j] = int8_t(mid[j]);
    const uint64_t nvb = uint64_t(1) << (n - t);
    // a few resident rounds of workgroups walk the tile pairs: a workgroup
    // per tile pair spends more on its launch than on its 2^t amplitudes
    const dim3 grid(unsigned(std::min<uint64_t>(nvb, uint64_t(svi_config().perm_workgroups))));
    const bool big = t > 10;
    if (s->dtype == SV_C128) {
        if (big)
            hipLaunchKernelGGL((k_bitperm_rl<c128, 12>), grid, dim3(kPermThreads), 0, s->stream,
                               static_cast<c128 *>(s->d), P, nvb);
        else
            hipLaunchKernelGGL((k_bitperm<c128, 10>), grid, dim3(kPermThreads), 0, s->stream,
                               static_cast<c128 *>(s->d), P, nvb);
    } else {
        if (big)
            hipLaunchKernelGGL((k_bitperm_rl<c64, 12>), grid, dim3(kPermThreads), 0, s->stream,
                               static_cast<c64 *>(s->d), P, nvb);
        else
            hipLaunchKernelGGL((k_bitperm<c64, 10>), grid, dim3(kPermThreads), 0, s->stream,
                               static_cast<c64 *>(s->d), P, nvb);
    }
    return hipGetLastError();
}
