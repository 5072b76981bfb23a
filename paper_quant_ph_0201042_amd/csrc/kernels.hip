// gfx950 kernels of the per-gate path: register set-up, one-qubit and
// controlled one-qubit gates, qubit swaps and FP64 reductions.
//
// Index arithmetic.  A gate on qubit q touches pairs of basis indices that
// differ only in bit b = n-1-q (sec. 2.2.1).  Instead of the paper's split of
// the matrix into blocks S_k handed to processors (with paired row chunks when
// blocks outnumber processors), every work item here is one pair (or one
// amplitude) named by a dense counter t; the basis index is t with zero bits
// inserted at the target position and at every control position, and the
// control bits then set to 1 (sec. 2.2.2: rows with a control bit 0 are left
// alone, so they are never visited).  One work item owns both halves of its
// pair, which removes the in-place hazard of the Parallelization paragraph of
// sec. 2.2.1 without any barrier; the kernel boundary is the per-gate
// barrier.
//
// Memory behaviour (the whole path is HBM bound: 14 flop per 32 bytes for
// complex128):
//   - b >= 6: k_pairs.  Lanes of a wavefront take consecutive t, so both the
//     i0 and the i1 streams are contiguous 64-amplitude runs (1 KiB for
//     complex128).  Each thread keeps PPT pairs in flight.
//   - b < 6: k_lowbit.  The partner of an amplitude lies in the same
//     64-amplitude run, so each lane loads one amplitude of a contiguous run
//     (fully coalesced) and fetches its partner with a cross-lane shuffle
//     (lane ^ 2^b); each lane writes back only its own amplitude.
//   - diagonal gates (Z, R_k, phases) only scale the target=1 amplitudes
//     (and the target=0 ones when u11 != 1): k_diag.
#include "sv_internal.h"

namespace {

template <typename T>
struct RealOf;
template <>
struct RealOf<double2> {
    using type = double;
};
template <>
struct RealOf<float2> {
    using type = float;
};

constexpr int kBlock = 256;

__device__ __forceinline__ uint64_t insert_zero(uint64_t t, int p) {
    const uint64_t lo = t & ((uint64_t(1) << p) - 1);
    return ((t & ~lo) << 1) | lo;
}

__device__ __forceinline__ uint64_t insert_zeros(uint64_t t, const BitSpec &s) {
    for (int i = 0; i < s.count; ++i) t = insert_zero(t, s.pos[i]);
    return t;
}

// r = m[o] * x + m[o+2] * y with m holding (re, im) pairs.
template <typename T, typename R>
__device__ __forceinline__ T mac2(const R *m, int o, T x, T y) {
    T r;
    r.x = m[o] * x.x - m[o + 1] * x.y + m[o + 2] * y.x - m[o + 3] * y.y;
    r.y = m[o] * x.y + m[o + 1] * x.x + m[o + 2] * y.y + m[o + 3] * y.x;
    return r;
}

template <typename T, typename R>
__device__ __forceinline__ T scale(R re, R im, T x) {
    T r;
    r.x = re * x.x - im * x.y;
    r.y = re * x.y + im * x.x;
    return r;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_reset(T *__restrict__ a, uint64_t N, uint64_t idx) {
    const uint64_t stride = uint64_t(gridDim.x) * kBlock;
    for (uint64_t j = uint64_t(blockIdx.x) * kBlock + threadIdx.x; j < N; j += stride) {
        T v;
        v.x = (j == idx) ? 1 : 0;
        v.y = 0;
        a[j] = v;
    }
}

// Dense 2x2 on pairs (i0, i0 | 2^b).  CTRL = false: no controls, a single
// inserted bit at b.  CTRL = true: zero bits inserted at every position in
// spec (target and controls, ascending), then the controls set.
template <typename T, int PPT, bool CTRL, bool PERM>
__global__ __launch_bounds__(kBlock) void k_pairs(T *__restrict__ a, uint64_t npairs, int b, uint64_t ctrl,
                                                  BitSpec spec, Mat2<typename RealOf<T>::type> u) {
    using R = typename RealOf<T>::type;
    const uint64_t tb = uint64_t(1) << b;
    const uint64_t base = uint64_t(blockIdx.x) * (kBlock * PPT) + threadIdx.x;
    uint64_t i0[PPT];
    T x[PPT], y[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const uint64_t t = base + uint64_t(k) * kBlock;
        i0[k] = CTRL ? (insert_zeros(t, spec) | ctrl) : insert_zero(t, b);
        if (t < npairs) {
            x[k] = a[i0[k]];
            y[k] = a[i0[k] | tb];
        }
    }
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const uint64_t t = base + uint64_t(k) * kBlock;
        if (t < npairs) {
            if (PERM) {
                a[i0[k]] = y[k];
                a[i0[k] | tb] = x[k];
            } else {
                const R *m = u.m;
                const T nx = mac2<T, R>(m, 0, x[k], y[k]);
                const T ny = mac2<T, R>(m, 4, x[k], y[k]);
                a[i0[k]] = nx;
                a[i0[k] | tb] = ny;
            }
        }
    }
}

template <typename T>
__device__ __forceinline__ T shfl_xor_c(T v, int m) {
    T r;
    r.x = __shfl_xor(v.x, m, 64);
    r.y = __shfl_xor(v.y, m, 64);
    return r;
}

// Target bit b < 6.  The state is walked in runs of 64 amplitudes, one run per
// wavefront step; run numbers are a dense counter c with the control bits at
// positions >= 6 inserted (hi, positions relative to bit 6) and set.  Control
// bits below 6 become a per-lane predicate.  Partner values travel by
// cross-lane shuffle, so both loads and stores are contiguous.
template <typename T, int CH, bool PERM>
__global__ __launch_bounds__(kBlock) void k_lowbit(T *__restrict__ a, uint64_t N, uint64_t nruns, int b,
                                                   uint64_t ctrl_lo, uint64_t ctrl_hi_runs, BitSpec hi,
                                                   Mat2<typename RealOf<T>::type> u) {
    using R = typename RealOf<T>::type;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int m = 1 << b;
    const bool upper = (lane >> b) & 1;
    uint64_t idx[CH];
    T x[CH];
    bool live[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        const uint64_t c = (uint64_t(blockIdx.x) * CH + k) * (kBlock / 64) + wave;
        live[k] = c < nruns;  // uniform over the wavefront
        const uint64_t run = insert_zeros(c, hi) | ctrl_hi_runs;
        idx[k] = (run << 6) | uint64_t(lane);
        x[k].x = 0;
        x[k].y = 0;
        if (live[k] && idx[k] < N) x[k] = a[idx[k]];
    }
#pragma unroll
    for (int k = 0; k < CH; ++k) {
        if (!live[k]) continue;
        const T p = shfl_xor_c(x[k], m);
        const bool act = idx[k] < N && (idx[k] & ctrl_lo) == ctrl_lo;
        if (!act) continue;
        T r;
        if (PERM) {
            r = p;
        } else {
            const R *mm = u.m;
            r = upper ? mac2<T, R>(mm, 4, p, x[k]) : mac2<T, R>(mm, 0, x[k], p);
        }
        a[idx[k]] = r;
    }
}

// Diagonal gate diag(u11, u22): amplitudes with the target bit 0 are scaled
// by u11 (when s0) and those with it 1 by u22 (when s1); an entry equal to 1
// is skipped, so R_k and Z read and write only the target=1 quarter or half.
// Counter t enumerates the target-and-controls subspace (all fixed bits
// inserted as zeros, then the controls set).
template <typename T, int PPT>
__global__ __launch_bounds__(kBlock) void k_diag(T *__restrict__ a, uint64_t count, int b, uint64_t ctrl,
                                                 BitSpec spec, Mat2<typename RealOf<T>::type> u, int s0, int s1) {
    using R = typename RealOf<T>::type;
    const uint64_t tb = uint64_t(1) << b;
    const uint64_t base = uint64_t(blockIdx.x) * (kBlock * PPT) + threadIdx.x;
    uint64_t i0[PPT];
    T y[PPT], x[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const uint64_t t = base + uint64_t(k) * kBlock;
        i0[k] = insert_zeros(t, spec) | ctrl;
        if (t < count) {
            if (s0) x[k] = a[i0[k]];
            if (s1) y[k] = a[i0[k] | tb];
        }
    }
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const uint64_t t = base + uint64_t(k) * kBlock;
        if (t < count) {
            if (s0) a[i0[k]] = scale<T, R>(u.m[0], u.m[1], x[k]);
            if (s1) a[i0[k] | tb] = scale<T, R>(u.m[6], u.m[7], y[k]);
        }
    }
}

// Exchange of qubit bits b1 < b2: amplitudes at i | 2^b1 and i | 2^b2 (i has
// both bits 0) trade places.
template <typename T, int PPT>
__global__ __launch_bounds__(kBlock) void k_swap(T *__restrict__ a, uint64_t count, int b1, int b2) {
    const uint64_t m1 = uint64_t(1) << b1, m2 = uint64_t(1) << b2;
    const uint64_t base = uint64_t(blockIdx.x) * (kBlock * PPT) + threadIdx.x;
    uint64_t i[PPT];
    T x[PPT], y[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const uint64_t t = base + uint64_t(k) * kBlock;
        i[k] = insert_zero(insert_zero(t, b1), b2);
        if (t < count) {
            x[k] = a[i[k] | m1];
            y[k] = a[i[k] | m2];
        }
    }
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const uint64_t t = base + uint64_t(k) * kBlock;
        if (t < count) {
            a[i[k] | m1] = y[k];
            a[i[k] | m2] = x[k];
        }
    }
}

// ------------------------------------------------------------ reductions
// Stage 1: block k sums elements [k*chunk, min((k+1)*chunk, count)) of the
// enumerated index space; each thread keeps four FP64 accumulators over a
// fixed strided walk, combined in a fixed order, then a fixed shared-memory
// tree.  Stage 2 sums the block partials with one block in the same way.  The
// order depends only on count, so results are bitwise reproducible.

template <int W>
__device__ __forceinline__ void block_tree(double (&v)[W], double *sh) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int w = 0; w < W; ++w) sh[w * SVI_RED_THREADS + tid] = v[w];
    __syncthreads();
    for (int s = SVI_RED_THREADS / 2; s > 0; s >>= 1) {
        if (tid < s) {
#pragma unroll
            for (int w = 0; w < W; ++w) sh[w * SVI_RED_THREADS + tid] += sh[w * SVI_RED_THREADS + tid + s];
        }
        __syncthreads();
    }
#pragma unroll
    for (int w = 0; w < W; ++w) v[w] = sh[w * SVI_RED_THREADS];
}

template <typename T>
__global__ __launch_bounds__(SVI_RED_THREADS) void k_prob1(const T *__restrict__ a, uint64_t count, uint64_t chunk,
                                                           BitSpec spec, uint64_t value, double *__restrict__ part) {
    __shared__ double sh[SVI_RED_THREADS];
    const uint64_t start = uint64_t(blockIdx.x) * chunk;
    const uint64_t end = min(start + chunk, count);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    uint64_t k = start + threadIdx.x;
    for (; k + 3 * SVI_RED_THREADS < end; k += 4 * SVI_RED_THREADS) {
        T v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint64_t e = k + uint64_t(u) * SVI_RED_THREADS;
            v[u] = a[spec.count ? (insert_zeros(e, spec) | value) : e];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double re = v[u].x, im = v[u].y;
            acc[u] += re * re + im * im;
        }
    }
    for (int u = 0; k < end; k += SVI_RED_THREADS, ++u) {
        const T v = a[spec.count ? (insert_zeros(k, spec) | value) : k];
        const double re = v.x, im = v.y;
        acc[u & 3] += re * re + im * im;
    }
    double s[1] = {(acc[0] + acc[1]) + (acc[2] + acc[3])};
    block_tree<1>(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

template <typename TA, typename TB>
__global__ __launch_bounds__(SVI_RED_THREADS) void k_inner1(const TA *__restrict__ a, const TB *__restrict__ b,
                                                            uint64_t count, uint64_t chunk, double *__restrict__ part) {
    __shared__ double sh[2 * SVI_RED_THREADS];
    const uint64_t start = uint64_t(blockIdx.x) * chunk;
    const uint64_t end = min(start + chunk, count);
    double re[4] = {0, 0, 0, 0}, im[4] = {0, 0, 0, 0};
    uint64_t k = start + threadIdx.x;
    for (; k + 3 * SVI_RED_THREADS < end; k += 4 * SVI_RED_THREADS) {
        TA va[4];
        TB vb[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            va[u] = a[k + uint64_t(u) * SVI_RED_THREADS];
            vb[u] = b[k + uint64_t(u) * SVI_RED_THREADS];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double ar = va[u].x, ai = va[u].y, br = vb[u].x, bi = vb[u].y;
            re[u] += ar * br + ai * bi;
            im[u] += ar * bi - ai * br;
        }
    }
    for (int u = 0; k < end; k += SVI_RED_THREADS, ++u) {
        const double ar = a[k].x, ai = a[k].y, br = b[k].x, bi = b[k].y;
        re[u & 3] += ar * br + ai * bi;
        im[u & 3] += ar * bi - ai * br;
    }
    double s[2] = {(re[0] + re[1]) + (re[2] + re[3]), (im[0] + im[1]) + (im[2] + im[3])};
    block_tree<2>(s, sh);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s[0];
        part[2 * blockIdx.x + 1] = s[1];
    }
}

// Sums W-wide partials of nparts blocks into out[0..W-1].
template <int W>
__global__ __launch_bounds__(SVI_RED_THREADS) void k_red2(const double *__restrict__ part, int nparts,
                                                          double *__restrict__ out) {
    __shared__ double sh[W * SVI_RED_THREADS];
    double v[W];
#pragma unroll
    for (int w = 0; w < W; ++w) v[w] = 0.0;
    for (int k = threadIdx.x; k < nparts; k += SVI_RED_THREADS) {
#pragma unroll
        for (int w = 0; w < W; ++w) v[w] += part[W * k + w];
    }
    block_tree<W>(v, sh);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int w = 0; w < W; ++w) out[w] = v[w];
    }
}

// ------------------------------------------------------------ helpers

uint64_t grid_for(uint64_t items, uint64_t per_block) { return (items + per_block - 1) / per_block; }

template <typename R>
Mat2<R> to_mat(const double U[8]) {
    Mat2<R> m;
    for (int i = 0; i < 8; ++i) m.m[i] = R(U[i]);
    return m;
}

// Ascending positions of the set bits of mask.
BitSpec bits_of(uint64_t mask) {
    BitSpec s{};
    s.count = 0;
    for (int p = 0; p < 64; ++p)
        if ((mask >> p) & 1) s.pos[s.count++] = uint8_t(p);
    return s;
}

template <typename T>
hipError_t launch_gate_t(sv_state *s, uint64_t ctrl, int q, const double U[8]) {
    using R = typename RealOf<T>::type;
    T *a = static_cast<T *>(s->d);
    const int n = s->n;
    const int b = n - 1 - q;
    const uint64_t N = uint64_t(1) << n;
    const int nc = __builtin_popcountll(ctrl);
    const GateClass gc = svi_classify(U);
    const Mat2<R> u = to_mat<R>(U);
    const BitSpec fixed = bits_of(ctrl | (uint64_t(1) << b));
    constexpr int PPT = 4;
    if (gc == GC_DIAG) {
        const int s0 = !(U[0] == 1.0 && U[1] == 0.0);
        const int s1 = !(U[6] == 1.0 && U[7] == 0.0);
        if (!s0 && !s1) return hipSuccess;  // identity
        const uint64_t count = N >> (nc + 1);
        hipLaunchKernelGGL((k_diag<T, PPT>), dim3(grid_for(count, kBlock * PPT)), dim3(kBlock), 0, s->stream, a,
                           count, b, ctrl, fixed, u, s0, s1);
        return hipGetLastError();
    }
    const bool perm = gc == GC_PERM;
    {
        if (b >= 6) {
            const uint64_t npairs = N >> (nc + 1);
            const dim3 grid(grid_for(npairs, kBlock * PPT));
            if (nc == 0) {
                if (perm)
                    hipLaunchKernelGGL((k_pairs<T, PPT, false, true>), grid, dim3(kBlock), 0, s->stream, a, npairs, b,
                                       ctrl, fixed, u);
                else
                    hipLaunchKernelGGL((k_pairs<T, PPT, false, false>), grid, dim3(kBlock), 0, s->stream, a, npairs,
                                       b, ctrl, fixed, u);
            } else {
                if (perm)
                    hipLaunchKernelGGL((k_pairs<T, PPT, true, true>), grid, dim3(kBlock), 0, s->stream, a, npairs, b,
                                       ctrl, fixed, u);
                else
                    hipLaunchKernelGGL((k_pairs<T, PPT, true, false>), grid, dim3(kBlock), 0, s->stream, a, npairs, b,
                                       ctrl, fixed, u);
            }
            return hipGetLastError();
        }
    }
    // b < 6: runs of 64 amplitudes, controls >= 6 enumerated, < 6 predicated
    const uint64_t ctrl_lo = ctrl & 63;
    const uint64_t ctrl_hi_runs = ctrl >> 6;
    const BitSpec hi = bits_of(ctrl_hi_runs);
    const int nhi = hi.count;
    const uint64_t nruns = (n >= 6) ? (uint64_t(1) << (n - 6 - nhi)) : 1;
    constexpr int CH = 4;
    const dim3 grid(grid_for(nruns, (kBlock / 64) * CH));
    if (perm)
        hipLaunchKernelGGL((k_lowbit<T, CH, true>), grid, dim3(kBlock), 0, s->stream, a, N, nruns, b, ctrl_lo,
                           ctrl_hi_runs, hi, u);
    else
        hipLaunchKernelGGL((k_lowbit<T, CH, false>), grid, dim3(kBlock), 0, s->stream, a, N, nruns, b, ctrl_lo,
                           ctrl_hi_runs, hi, u);
    return hipGetLastError();
}

}  // namespace

hipError_t svi_launch_reset(sv_state *s, uint64_t idx) {
    const uint64_t N = uint64_t(1) << s->n;
    const uint64_t blocks = std::min<uint64_t>(grid_for(N, kBlock), 65536);
    if (s->dtype == SV_C128)
        hipLaunchKernelGGL((k_reset<double2>), dim3(blocks), dim3(kBlock), 0, s->stream,
                           static_cast<double2 *>(s->d), N, idx);
    else
        hipLaunchKernelGGL((k_reset<float2>), dim3(blocks), dim3(kBlock), 0, s->stream, static_cast<float2 *>(s->d),
                           N, idx);
    return hipGetLastError();
}

hipError_t svi_launch_gate(sv_state *s, uint64_t ctrl, int q, const double U[8]) {
    return s->dtype == SV_C128 ? launch_gate_t<double2>(s, ctrl, q, U) : launch_gate_t<float2>(s, ctrl, q, U);
}

hipError_t svi_launch_swap(sv_state *s, int q1, int q2) {
    if (q1 == q2) return hipSuccess;
    int b1 = s->n - 1 - q1, b2 = s->n - 1 - q2;
    if (b1 > b2) std::swap(b1, b2);
    const uint64_t count = uint64_t(1) << (s->n - 2);
    constexpr int PPT = 4;
    const dim3 grid(grid_for(count, kBlock * PPT));
    if (s->dtype == SV_C128)
        hipLaunchKernelGGL((k_swap<double2, PPT>), grid, dim3(kBlock), 0, s->stream, static_cast<double2 *>(s->d),
                           count, b1, b2);
    else
        hipLaunchKernelGGL((k_swap<float2, PPT>), grid, dim3(kBlock), 0, s->stream, static_cast<float2 *>(s->d),
                           count, b1, b2);
    return hipGetLastError();
}

namespace {
// Fixed partition of count elements over at most SVI_RED_BLOCKS blocks.
void red_geometry(uint64_t count, uint64_t *chunk, int *blocks) {
    uint64_t per = std::max<uint64_t>(uint64_t(4) * SVI_RED_THREADS, (count + SVI_RED_BLOCKS - 1) / SVI_RED_BLOCKS);
    *chunk = per;
    *blocks = int((count + per - 1) / per);
    if (*blocks < 1) *blocks = 1;
}
}  // namespace

hipError_t svi_launch_prob(sv_state *s, uint64_t mask, uint64_t value) {
    const int nm = __builtin_popcountll(mask);
    const uint64_t count = uint64_t(1) << (s->n - nm);
    uint64_t chunk;
    int blocks;
    red_geometry(count, &chunk, &blocks);
    const BitSpec spec = bits_of(mask);
    double *part = s->d_red;
    double *out = s->d_red + 2 * SVI_RED_BLOCKS;
    if (s->dtype == SV_C128)
        hipLaunchKernelGGL((k_prob1<double2>), dim3(blocks), dim3(SVI_RED_THREADS), 0, s->stream,
                           static_cast<const double2 *>(s->d), count, chunk, spec, value, part);
    else
        hipLaunchKernelGGL((k_prob1<float2>), dim3(blocks), dim3(SVI_RED_THREADS), 0, s->stream,
                           static_cast<const float2 *>(s->d), count, chunk, spec, value, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_red2<1>), dim3(1), dim3(SVI_RED_THREADS), 0, s->stream, part, blocks, out);
    return hipGetLastError();
}

hipError_t svi_launch_inner(sv_state *a, sv_state *b, hipStream_t st) {
    const uint64_t count = uint64_t(1) << a->n;
    uint64_t chunk;
    int blocks;
    red_geometry(count, &chunk, &blocks);
    double *part = b->d_red;
    double *out = b->d_red + 2 * SVI_RED_BLOCKS;
    const dim3 g(blocks), t(SVI_RED_THREADS);
    if (a->dtype == SV_C128 && b->dtype == SV_C128)
        hipLaunchKernelGGL((k_inner1<double2, double2>), g, t, 0, st, static_cast<const double2 *>(a->d),
                           static_cast<const double2 *>(b->d), count, chunk, part);
    else if (a->dtype == SV_C128)
        hipLaunchKernelGGL((k_inner1<double2, float2>), g, t, 0, st, static_cast<const double2 *>(a->d),
                           static_cast<const float2 *>(b->d), count, chunk, part);
    else if (b->dtype == SV_C128)
        hipLaunchKernelGGL((k_inner1<float2, double2>), g, t, 0, st, static_cast<const float2 *>(a->d),
                           static_cast<const double2 *>(b->d), count, chunk, part);
    else
        hipLaunchKernelGGL((k_inner1<float2, float2>), g, t, 0, st, static_cast<const float2 *>(a->d),
                           static_cast<const float2 *>(b->d), count, chunk, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_red2<2>), dim3(1), dim3(SVI_RED_THREADS), 0, st, part, blocks, out);
    return hipGetLastError();
}
