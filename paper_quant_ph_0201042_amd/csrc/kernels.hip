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
// Memory behaviour.  The per-gate path is HBM bound (complex128: 14 flop per
// 32 bytes moved).  Measured on MI355X at n = 30, what decides the achieved
// bandwidth is the access footprint, not the arithmetic:
//   - nontemporal loads and stores (the state never fits in cache);
//   - one pair per thread, 256 threads per workgroup;
//   - for complex128, each workgroup takes two 256-pair slices of the counter
//     space split at counter bit 11 ("NS = 2"), which keeps 6.0-6.4 TB/s for
//     every target bit; target bits 11 and 12 do best with one slice.
// Kernels:
//   - k_pairs, target bit b >= 6: lanes take consecutive counters, so both
//     halves of the pairs are contiguous runs.
//   - k_lowbit, b < 6: the partner lies in the same 64-amplitude run; each
//     lane loads one amplitude of a contiguous run, fetches its partner by a
//     cross-lane shuffle (lane ^ 2^b) and writes back only its own amplitude.
//   - k_diag: diagonal gates (Z, R_k, phases) scale only the amplitudes whose
//     factor is not 1.
#include "device_common.h"

using namespace svd;

namespace {

constexpr int kBlock = 256;
constexpr int kSliceBit = 11;  // counter bit separating the two slices of a workgroup

// A dispatch holds at most 2^32 work-items, so kernels walk "virtual
// blocks" vb = blockIdx.x, blockIdx.x + gridDim.x, ... up to nvb; launches
// cap the grid at kMaxGrid workgroups (one round for registers up to about
// 30 qubits).
constexpr uint64_t kMaxGrid = uint64_t(1) << 20;

// Counter of slice 0 of virtual block vb (NS slices of kBlock counters).
template <int NS>
__device__ __forceinline__ uint64_t slice_base(uint64_t vb, int s) {
    uint64_t c0 = vb * kBlock;
    if (NS == 2) c0 = insert_zero(c0, s);
    return c0 + threadIdx.x;
}

// Virtual block order with the low tk bits of vb moved to the top of its
// vbits bits (a bijection on [0, 2^vbits)): workgroups that run together
// then lie 2^(vbits - tk) blocks apart.  tk = 0 keeps the plain order.
__device__ __forceinline__ uint64_t spread_vb(uint64_t vb, int tk, int vbits) {
    if (tk == 0) return vb;
    return (vb >> tk) | ((vb & ((uint64_t(1) << tk) - 1)) << (vbits - tk));
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_reset(T *__restrict__ a, uint64_t N, uint64_t idx, uint64_t nvb) {
    for (uint64_t vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
        const uint64_t j = vb * kBlock + threadIdx.x;
        if (j < N) {
            T v;
            v.x = (j == idx) ? 1 : 0;
            v.y = 0;
            stnt(v, a + j);
        }
    }
}

// VEC consecutive amplitudes (along index bit 0) as one access: complex64
// kernels move two amplitudes (16 bytes) per lane, complex128 one.
template <typename T, int VEC>
struct VecOf;
template <typename T>
struct VecOf<T, 1> {
    using type = T;
    static __device__ __forceinline__ T get(const type &v, int) { return v; }
    static __device__ __forceinline__ void put(type &v, int, T x) { v = x; }
};
template <>
struct VecOf<c64, 2> {
    typedef float type __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ c64 get(const type &v, int i) { return i ? c64{v.z, v.w} : c64{v.x, v.y}; }
    static __device__ __forceinline__ void put(type &v, int i, c64 x) {
        if (i) {
            v.z = x.x;
            v.w = x.y;
        } else {
            v.x = x.x;
            v.y = x.y;
        }
    }
};

template <typename T, int VEC>
__device__ __forceinline__ typename VecOf<T, VEC>::type ldv(const T *p) {
    return ldnt(reinterpret_cast<const typename VecOf<T, VEC>::type *>(p));
}
template <typename T, int VEC>
__device__ __forceinline__ void stv(typename VecOf<T, VEC>::type v, T *p) {
    stnt(v, reinterpret_cast<typename VecOf<T, VEC>::type *>(p));
}
// The same with the cache's default policy: for a target bit inside a
// 128-byte line both halves of a pair share lines, and the second access
// must find the line the first one brought in.
template <typename T, int VEC>
__device__ __forceinline__ typename VecOf<T, VEC>::type ldv_c(const T *p) {
    return *reinterpret_cast<const typename VecOf<T, VEC>::type *>(p);
}
template <typename T, int VEC>
__device__ __forceinline__ void stv_c(typename VecOf<T, VEC>::type v, T *p) {
    *reinterpret_cast<typename VecOf<T, VEC>::type *>(p) = v;
}

// Dense 2x2 (or an exact NOT when PERM) on pairs (i0, i0 | 2^b), b >= 6.
// Work item t covers VEC pairs at i0 + v: the counter with zero bits
// inserted at every position of spec (the target and the controls at or
// above the cache-line bits), those controls then set.  Controls below the
// line bits (ctrl_lo) are a predicate: a pair that fails it is written back
// unchanged, so every touched 128-byte line is written whole.
template <typename T, int NS, int VEC, bool PERM, bool CACHED = false>
__global__ __launch_bounds__(kBlock) void k_pairs(T *__restrict__ a, uint64_t count, int b, uint64_t ctrl_hi,
                                                  uint64_t ctrl_lo, BitSpec spec, int s,
                                                  Mat2<typename RealOf<T>::type> u, uint64_t nvb, int tk, int vbits) {
    using R = typename RealOf<T>::type;
    using V = VecOf<T, VEC>;
    const uint64_t tb = uint64_t(1) << b;
    for (uint64_t vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
    const uint64_t c0 = slice_base<NS>(spread_vb(vb, tk, vbits), s);
    uint64_t i0[NS];
    typename V::type x[NS], y[NS];
#pragma unroll
    for (int h = 0; h < NS; ++h) {
        const uint64_t t = c0 + (h ? (uint64_t(1) << s) : 0);
        i0[h] = insert_zeros(t * VEC, spec) | ctrl_hi;
        if (t < count) {
            x[h] = CACHED ? ldv_c<T, VEC>(a + i0[h]) : ldv<T, VEC>(a + i0[h]);
            y[h] = CACHED ? ldv_c<T, VEC>(a + (i0[h] | tb)) : ldv<T, VEC>(a + (i0[h] | tb));
        }
    }
#pragma unroll
    for (int h = 0; h < NS; ++h) {
        const uint64_t t = c0 + (h ? (uint64_t(1) << s) : 0);
        if (t >= count) continue;
        typename V::type xo = x[h], yo = y[h];
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            if (((i0[h] + v) & ctrl_lo) != ctrl_lo) continue;
            const T xv = V::get(x[h], v), yv = V::get(y[h], v);
            if (PERM) {
                V::put(xo, v, yv);
                V::put(yo, v, xv);
            } else {
                V::put(xo, v, mac2<T, R>(u.m, 0, xv, yv));
                V::put(yo, v, mac2<T, R>(u.m, 4, xv, yv));
            }
        }
        if (CACHED) {
            stv_c<T, VEC>(xo, a + i0[h]);
            stv_c<T, VEC>(yo, a + (i0[h] | tb));
        } else {
            stv<T, VEC>(xo, a + i0[h]);
            stv<T, VEC>(yo, a + (i0[h] | tb));
        }
    }
    }
}

// Target bit b < 6.  A wavefront covers 64 * VEC amplitudes: VEC along bit
// 0 inside a lane, then the lane bits, which are the lowest positions that
// are not controls at or above the cache-line bits (lanebit[]).  The runs
// (wavefront index c) enumerate the remaining positions with those controls
// inserted and set (run_spec holds every lane-bit and control position).
// The partner of a lane's amplitude is in the same lane (b = 0 with VEC = 2)
// or in lane ^ pmask.  Controls below the line bits are a per-amplitude
// predicate with the failing amplitudes written back unchanged.
// Each wavefront takes U consecutive runs per trip and issues all their
// loads before the first shuffle, so a lane keeps U accesses in flight (one
// run at a time left the dense low-bit gates at 0.46 of peak).
template <typename T, int VEC, bool PERM, int U>
__global__ __launch_bounds__(kBlock) void k_lowbit(T *__restrict__ a, uint64_t N, uint64_t nruns, int b,
                                                   uint64_t ctrl_lo, uint64_t ctrl_hi, BitSpec run_spec,
                                                   BitSpec lanebit, int pmask, Mat2<typename RealOf<T>::type> u,
                                                   uint64_t nvb) {
    using R = typename RealOf<T>::type;
    using V = VecOf<T, VEC>;
    const int lane = threadIdx.x & 63;
    // the lane's part of the index: its 6 lane bits deposited at their positions
    uint64_t off = 0;
    for (int i = 0; i < 6; ++i) off |= uint64_t((lane >> i) & 1) << lanebit.pos[i];
    const uint64_t tb = uint64_t(1) << b;
    for (uint64_t vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
    const uint64_t c0 = (vb * (kBlock / 64) + (threadIdx.x >> 6)) * U;
    uint64_t idx[U];
    typename V::type x[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
        idx[k] = insert_zeros(c0 + k, run_spec) | ctrl_hi | off;
        for (int v = 0; v < VEC; ++v) V::put(x[k], v, T{0, 0});
        if (c0 + k < nruns && idx[k] < N) x[k] = ldv<T, VEC>(a + idx[k]);
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
    if (c0 + k >= nruns) continue;  // uniform over the wavefront
    typename V::type r = x[k];
    if (VEC == 2 && b == 0) {
        // both halves of the pair in this lane
        const T x0 = V::get(x[k], 0), x1 = V::get(x[k], 1);
        if ((idx[k] & ctrl_lo) == ctrl_lo) {
            if (PERM) {
                V::put(r, 0, x1);
                V::put(r, 1, x0);
            } else {
                V::put(r, 0, mac2<T, R>(u.m, 0, x0, x1));
                V::put(r, 1, mac2<T, R>(u.m, 4, x0, x1));
            }
        }
    } else {
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            const T xv = V::get(x[k], v);
            const T p = shfl_xor_c(xv, pmask);
            const uint64_t iv = idx[k] + uint64_t(v);
            if ((iv & ctrl_lo) != ctrl_lo) continue;
            if (PERM)
                V::put(r, v, p);
            else
                V::put(r, v, (iv & tb) ? mac2<T, R>(u.m, 4, p, xv) : mac2<T, R>(u.m, 0, xv, p));
        }
    }
    if (idx[k] < N) stv<T, VEC>(r, a + idx[k]);
    }
    }
}

// Diagonal gate diag(u11, u22) on the amplitudes with (j & M) == Vv (M: the
// controls, and the target when only one entry differs from 1).  Work item
// t covers VEC amplitudes at idx + v: the counter with zero bits inserted at
// the positions of M at or above the cache-line bits (spec), those set to
// their value (v_hi).  Positions of M below the line bits are a predicate
// (m_lo, v_lo); every enumerated amplitude is written back, so lines are
// written whole.  An entry equal to 1 is not applied (s0, s1).
template <typename T, int NS, int VEC>
__global__ __launch_bounds__(kBlock) void k_diag(T *__restrict__ a, uint64_t count, int b, uint64_t v_hi,
                                                 uint64_t m_lo, uint64_t v_lo, BitSpec spec, int s,
                                                 Mat2<typename RealOf<T>::type> u, int s0, int s1, uint64_t nvb,
                                                 int tk, int vbits) {
    using R = typename RealOf<T>::type;
    using V = VecOf<T, VEC>;
    for (uint64_t vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
    const uint64_t c0 = slice_base<NS>(spread_vb(vb, tk, vbits), s);
    uint64_t i0[NS];
    typename V::type x[NS];
#pragma unroll
    for (int h = 0; h < NS; ++h) {
        const uint64_t t = c0 + (h ? (uint64_t(1) << s) : 0);
        i0[h] = insert_zeros(t * VEC, spec) | v_hi;
        if (t < count) x[h] = ldv<T, VEC>(a + i0[h]);
    }
#pragma unroll
    for (int h = 0; h < NS; ++h) {
        const uint64_t t = c0 + (h ? (uint64_t(1) << s) : 0);
        if (t >= count) continue;
        typename V::type r = x[h];
#pragma unroll
        for (int v = 0; v < VEC; ++v) {
            const uint64_t iv = i0[h] + uint64_t(v);
            if ((iv & m_lo) != v_lo) continue;
            const bool hi = (iv >> b) & 1;
            if (hi ? !s1 : !s0) continue;
            V::put(r, v, hi ? cscale<T, R>(u.m[6], u.m[7], V::get(r, v)) : cscale<T, R>(u.m[0], u.m[1], V::get(r, v)));
        }
        stv<T, VEC>(r, a + i0[h]);
    }
    }
}

// Exchange of qubit bits b1 < b2: amplitudes at i | 2^b1 and i | 2^b2 (i with
// both bits 0) trade places.
template <typename T, int NS>
__global__ __launch_bounds__(kBlock) void k_swap(T *__restrict__ a, uint64_t count, int b1, int b2, int s,
                                                 uint64_t nvb) {
    const uint64_t m1 = uint64_t(1) << b1, m2 = uint64_t(1) << b2;
    for (uint64_t vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
    const uint64_t c0 = slice_base<NS>(vb, s);
    uint64_t i[NS];
    T x[NS], y[NS];
#pragma unroll
    for (int h = 0; h < NS; ++h) {
        const uint64_t t = c0 + (h ? (uint64_t(1) << s) : 0);
        i[h] = insert_zero(insert_zero(t, b1), b2);
        if (t < count) {
            x[h] = ldnt(a + (i[h] | m1));
            y[h] = ldnt(a + (i[h] | m2));
        }
    }
#pragma unroll
    for (int h = 0; h < NS; ++h) {
        const uint64_t t = c0 + (h ? (uint64_t(1) << s) : 0);
        if (t < count) {
            stnt(y[h], a + (i[h] | m1));
            stnt(x[h], a + (i[h] | m2));
        }
    }
    }
}

// Projection onto the basis states with (j & mask) == value, scaled by
// `scale` (1/sqrt of their total weight): the other amplitudes become 0
// without being read.
template <typename T>
__global__ __launch_bounds__(256) void k_collapse(T *__restrict__ a, uint64_t count, uint64_t mask, uint64_t value,
                                                  typename RealOf<T>::type scale, uint64_t nvb) {
    for (uint64_t vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
        const uint64_t j = vb * 256 + threadIdx.x;
        if (j >= count) continue;
        T v;
        if ((j & mask) == value) {
            v = ldnt(a + j);
            v.x *= scale;
            v.y *= scale;
        } else {
            v.x = 0;
            v.y = 0;
        }
        stnt(v, a + j);
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
    for (int st = SVI_RED_THREADS / 2; st > 0; st >>= 1) {
        if (tid < st) {
#pragma unroll
            for (int w = 0; w < W; ++w) sh[w * SVI_RED_THREADS + tid] += sh[w * SVI_RED_THREADS + tid + st];
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
        for (int w = 0; w < 4; ++w) {
            const uint64_t e = k + uint64_t(w) * SVI_RED_THREADS;
            v[w] = ldnt(a + (spec.count ? (insert_zeros(e, spec) | value) : e));
        }
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const double re = v[w].x, im = v[w].y;
            acc[w] += re * re + im * im;
        }
    }
    for (int w = 0; k < end; k += SVI_RED_THREADS, ++w) {
        const T v = ldnt(a + (spec.count ? (insert_zeros(k, spec) | value) : k));
        const double re = v.x, im = v.y;
        acc[w & 3] += re * re + im * im;
    }
    double sum[1] = {(acc[0] + acc[1]) + (acc[2] + acc[3])};
    block_tree<1>(sum, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = sum[0];
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
        for (int w = 0; w < 4; ++w) {
            va[w] = ldnt(a + k + uint64_t(w) * SVI_RED_THREADS);
            vb[w] = ldnt(b + k + uint64_t(w) * SVI_RED_THREADS);
        }
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const double ar = va[w].x, ai = va[w].y, br = vb[w].x, bi = vb[w].y;
            re[w] += ar * br + ai * bi;
            im[w] += ar * bi - ai * br;
        }
    }
    for (int w = 0; k < end; k += SVI_RED_THREADS, ++w) {
        const TA va = ldnt(a + k);
        const TB vb = ldnt(b + k);
        const double ar = va.x, ai = va.y, br = vb.x, bi = vb.y;
        re[w & 3] += ar * br + ai * bi;
        im[w & 3] += ar * bi - ai * br;
    }
    double sum[2] = {(re[0] + re[1]) + (re[2] + re[3]), (im[0] + im[1]) + (im[2] + im[3])};
    block_tree<2>(sum, sh);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sum[0];
        part[2 * blockIdx.x + 1] = sum[1];
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

// ------------------------------------------------------------ host side

uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
dim3 capped(uint64_t nvb) { return dim3(unsigned(nvb < kMaxGrid ? nvb : kMaxGrid)); }

template <typename R>
Mat2<R> to_mat(const double U[8]) {
    Mat2<R> m;
    for (int i = 0; i < 8; ++i) m.m[i] = R(U[i]);
    return m;
}

}  // namespace

BitSpec svi_bits_of(uint64_t mask) {
    BitSpec s{};
    s.count = 0;
    for (int p = 0; p < 64; ++p)
        if ((mask >> p) & 1) s.pos[s.count++] = uint8_t(p);
    return s;
}

namespace {

// Slice count for a counter space of `count` work items: two slices split at
// kSliceBit for complex128 when the space is large enough, else one.
template <typename T>
int slices_for(uint64_t count, int b, bool ctrl) {
    if (sizeof(T) != 16) return 1;
    if (count < (uint64_t(1) << (kSliceBit + 1))) return 1;
    if (!ctrl && (b == 11 || b == 12)) return 1;
    return 2;
}

// Index bits below this hold one 128-byte cache line (8 complex128 or 16
// complex64 amplitudes): a fixed bit there leaves every line touched.
template <typename T>
constexpr int line_bits() {
    return sizeof(T) == 16 ? 3 : 4;
}

// Block-order spread (spread_vb) of a pair or diagonal launch.  With fixed
// index bits (controls, or a diagonal gate's target whose other entry is 1)
// at byte address bits 10..12 or 20..21, the workgroups that run together
// in plain order reach only part of the memory channels: on MI355X a
// controlled phase with both its bits there ran at 0.55-0.63 of the HBM
// peak, CNOT with its control there at 0.58-0.61, and 0.70-0.80 with the
// low 4 bits of the block index moved to its top (no other gate class or
// bit changed by more than noise).  Returns tk (0: plain order) and sets
// vbits = log2(nvb); the spread needs nvb a power of two above 2^tk.
template <typename T>
int spread_bits(uint64_t fixed_hi, uint64_t nvb, int &vbits) {
    vbits = 0;
    while ((uint64_t(1) << vbits) < nvb) ++vbits;
    const int k = svi_config().gate_spread_bits;
    constexpr int kAmpBits = sizeof(T) == 16 ? 4 : 3;  // log2 of the bytes per amplitude
    const uint64_t window = ((uint64_t(7) << 10) | (uint64_t(3) << 20)) >> kAmpBits;  // at byte bits 10..12, 20..21
    if (k == 0 || !(fixed_hi & window) || (nvb & (nvb - 1)) != 0 || vbits <= k) return 0;
    return k;
}

template <typename T>
hipError_t launch_gate_t(sv_state *s, uint64_t ctrl, int q, const double U[8]) {
    using R = typename RealOf<T>::type;
    T *a = static_cast<T *>(s->d);
    const int n = s->n;
    const int b = n - 1 - q;
    const uint64_t N = uint64_t(1) << n;
    const GateClass gc = svi_classify(U);
    const Mat2<R> u = to_mat<R>(U);
    const dim3 blk(kBlock);
    const uint64_t lomask = (uint64_t(1) << line_bits<T>()) - 1;
    // complex64 moves two amplitudes per lane (16-byte accesses)
    constexpr int VEC = sizeof(T) == 8 ? 2 : 1;
    if (gc == GC_DIAG) {
        const int s0 = !(U[0] == 1.0 && U[1] == 0.0);
        const int s1 = !(U[6] == 1.0 && U[7] == 0.0);
        if (!s0 && !s1) return hipSuccess;  // identity
        const uint64_t tb = uint64_t(1) << b;
        const uint64_t M = ctrl | (s0 != s1 ? tb : 0);
        const uint64_t Vv = ctrl | (s1 && !s0 ? tb : 0);
        const uint64_t m_hi = M & ~lomask;
        const BitSpec spec = svi_bits_of(m_hi);
        const uint64_t count = (N >> spec.count) / VEC;
        // complex64 moves 16 bytes per access: two slices per work item keep
        // two accesses in flight per lane (one left it at 0.65 of peak)
        const int ns = VEC == 2 ? (count >= (uint64_t(1) << (kSliceBit + 1)) ? 2 : 1) : slices_for<T>(count, b, true);
        const uint64_t nvb = ceil_div(count, uint64_t(kBlock) * ns);
        int vbits = 0;
        const int tk = spread_bits<T>(m_hi, nvb, vbits);
        if (VEC == 2 && ns == 2)
            hipLaunchKernelGGL((k_diag<T, 2, VEC>), capped(nvb), blk, 0, s->stream, a, count, b, Vv & m_hi,
                               M & lomask, Vv & lomask, spec, kSliceBit, u, s0, s1, nvb, tk, vbits);
        else if (VEC == 2)
            hipLaunchKernelGGL((k_diag<T, 1, VEC>), capped(nvb), blk, 0, s->stream, a, count, b, Vv & m_hi,
                               M & lomask, Vv & lomask, spec, kSliceBit, u, s0, s1, nvb, tk, vbits);
        else if (ns == 2)
            hipLaunchKernelGGL((k_diag<T, 2, 1>), capped(nvb), blk, 0, s->stream, a, count, b, Vv & m_hi, M & lomask,
                               Vv & lomask, spec, kSliceBit, u, s0, s1, nvb, tk, vbits);
        else
            hipLaunchKernelGGL((k_diag<T, 1, 1>), capped(nvb), blk, 0, s->stream, a, count, b, Vv & m_hi, M & lomask,
                               Vv & lomask, spec, kSliceBit, u, s0, s1, nvb, tk, vbits);
        return hipGetLastError();
    }
    const bool perm = gc == GC_PERM;
    const uint64_t ctrl_hi = ctrl & ~lomask, ctrl_lo = ctrl & lomask;
    if (VEC == 2 && b == 0 && svi_config().gate_pairs_min_bit == 0) {
        // complex64 target bit 0: both halves of a pair are neighbours, so
        // the pair kernel takes one amplitude per access (8 bytes)
        const BitSpec spec = svi_bits_of(ctrl_hi | 1);
        const uint64_t count = N >> spec.count;
        const uint64_t nvb = ceil_div(count, uint64_t(kBlock));
        const bool cached = svi_config().gate_cached_low != 0;
        int vbits = 0;
        const int tk = spread_bits<T>(ctrl_hi, nvb, vbits);
#define SV_LAUNCH_PAIRS0(P, C)                                                                                        \
    hipLaunchKernelGGL((k_pairs<T, 1, 1, P, C>), capped(nvb), blk, 0, s->stream, a, count, 0, ctrl_hi, ctrl_lo, spec, \
                       kSliceBit, u, nvb, tk, vbits)
        if (perm) {
            if (cached) SV_LAUNCH_PAIRS0(true, true); else SV_LAUNCH_PAIRS0(true, false);
        } else {
            if (cached) SV_LAUNCH_PAIRS0(false, true); else SV_LAUNCH_PAIRS0(false, false);
        }
#undef SV_LAUNCH_PAIRS0
        return hipGetLastError();
    }
    if (b >= std::max(svi_config().gate_pairs_min_bit, VEC == 2 ? 1 : 0)) {
        const BitSpec spec = svi_bits_of(ctrl_hi | (uint64_t(1) << b));
        const uint64_t count = (N >> spec.count) / VEC;
        // a target bit inside a 128-byte line: both halves of a pair share
        // lines (cached accesses, gate_cached_low; one slice)
        const bool cached = b < line_bits<T>() && svi_config().gate_cached_low != 0;
        const int ns = (VEC == 2 || cached) ? 1 : slices_for<T>(count, b, ctrl != 0);
        const uint64_t nvb = ceil_div(count, uint64_t(kBlock) * ns);
        const dim3 grid = capped(nvb);
        int vbits = 0;
        const int tk = spread_bits<T>(ctrl_hi, nvb, vbits);
#define SV_LAUNCH_PAIRS(NS, P, C)                                                                                     \
    hipLaunchKernelGGL((k_pairs<T, NS, VEC, P, C>), grid, blk, 0, s->stream, a, count, b, ctrl_hi, ctrl_lo, spec,     \
                       kSliceBit, u, nvb, tk, vbits)
        if (cached) {
            if (perm) SV_LAUNCH_PAIRS(1, true, true); else SV_LAUNCH_PAIRS(1, false, true);
        } else if (ns == 2) {
            if (perm) SV_LAUNCH_PAIRS(2, true, false); else SV_LAUNCH_PAIRS(2, false, false);
        } else {
            if (perm) SV_LAUNCH_PAIRS(1, true, false); else SV_LAUNCH_PAIRS(1, false, false);
        }
#undef SV_LAUNCH_PAIRS
        return hipGetLastError();
    }
    // b < 6: lane bits are the lowest positions that are not high controls
    // (after bit 0 inside the lane for complex64)
    const int vbits = VEC == 2 ? 1 : 0;
    BitSpec lanebit{};
    lanebit.count = 6;
    uint64_t lanemask = 0;
    int pmask = 0, k = 0;
    for (int p = vbits; k < 6; ++p) {
        if ((ctrl_hi >> p) & 1) continue;
        lanebit.pos[k] = uint8_t(p);
        lanemask |= uint64_t(1) << p;
        if (p == b) pmask = 1 << k;
        ++k;
    }
    if (vbits && b == 0) pmask = 0;
    const BitSpec run_spec = svi_bits_of(lanemask | ctrl_hi | (vbits ? 1 : 0));
    const int used = run_spec.count;
    const uint64_t nruns = n > used ? (uint64_t(1) << (n - used)) : 1;
    constexpr int RU = 4;  // runs per wavefront and trip
    const uint64_t rvb = ceil_div(nruns, (kBlock / 64) * RU);
    const dim3 rgrid = capped(rvb);
    if (perm)
        hipLaunchKernelGGL((k_lowbit<T, VEC, true, RU>), rgrid, blk, 0, s->stream, a, N, nruns, b, ctrl_lo, ctrl_hi,
                           run_spec, lanebit, pmask, u, rvb);
    else
        hipLaunchKernelGGL((k_lowbit<T, VEC, false, RU>), rgrid, blk, 0, s->stream, a, N, nruns, b, ctrl_lo, ctrl_hi,
                           run_spec, lanebit, pmask, u, rvb);
    return hipGetLastError();
}

}  // namespace

hipError_t svi_launch_reset(sv_state *s, uint64_t idx) {
    const uint64_t N = uint64_t(1) << s->n;
    const uint64_t nvb = ceil_div(N, kBlock);
    if (s->dtype == SV_C128)
        hipLaunchKernelGGL((k_reset<c128>), capped(nvb), dim3(kBlock), 0, s->stream, static_cast<c128 *>(s->d), N, idx,
                           nvb);
    else
        hipLaunchKernelGGL((k_reset<c64>), capped(nvb), dim3(kBlock), 0, s->stream, static_cast<c64 *>(s->d), N, idx,
                           nvb);
    return hipGetLastError();
}

hipError_t svi_launch_reset_ptr(void *d, int dtype, uint64_t N, uint64_t idx, hipStream_t st) {
    const uint64_t nvb = ceil_div(N, kBlock);
    if (dtype == SV_C128)
        hipLaunchKernelGGL((k_reset<c128>), capped(nvb), dim3(kBlock), 0, st, static_cast<c128 *>(d), N, idx, nvb);
    else
        hipLaunchKernelGGL((k_reset<c64>), capped(nvb), dim3(kBlock), 0, st, static_cast<c64 *>(d), N, idx, nvb);
    return hipGetLastError();
}

hipError_t svi_launch_gate(sv_state *s, uint64_t ctrl, int q, const double U[8]) {
    return s->dtype == SV_C128 ? launch_gate_t<c128>(s, ctrl, q, U) : launch_gate_t<c64>(s, ctrl, q, U);
}

hipError_t svi_launch_swap(sv_state *s, int q1, int q2) {
    if (q1 == q2) return hipSuccess;
    int b1 = s->n - 1 - q1, b2 = s->n - 1 - q2;
    if (b1 > b2) std::swap(b1, b2);
    const uint64_t count = uint64_t(1) << (s->n - 2);
    if (s->dtype == SV_C128) {
        const int ns = slices_for<c128>(count, -1, true);
        const uint64_t nvb = ceil_div(count, uint64_t(kBlock) * ns);
        if (ns == 2)
            hipLaunchKernelGGL((k_swap<c128, 2>), capped(nvb), dim3(kBlock), 0, s->stream, static_cast<c128 *>(s->d),
                               count, b1, b2, kSliceBit, nvb);
        else
            hipLaunchKernelGGL((k_swap<c128, 1>), capped(nvb), dim3(kBlock), 0, s->stream, static_cast<c128 *>(s->d),
                               count, b1, b2, kSliceBit, nvb);
    } else {
        const uint64_t nvb = ceil_div(count, kBlock);
        hipLaunchKernelGGL((k_swap<c64, 1>), capped(nvb), dim3(kBlock), 0, s->stream, static_cast<c64 *>(s->d), count,
                           b1, b2, kSliceBit, nvb);
    }
    return hipGetLastError();
}

namespace {
// Fixed partition of count elements over at most SVI_RED_BLOCKS blocks.
void red_geometry(uint64_t count, uint64_t *chunk, int *blocks) {
    const uint64_t per =
        std::max<uint64_t>(uint64_t(4) * SVI_RED_THREADS, (count + SVI_RED_BLOCKS - 1) / SVI_RED_BLOCKS);
    *chunk = per;
    *blocks = int((count + per - 1) / per);
    if (*blocks < 1) *blocks = 1;
}
}  // namespace

hipError_t svi_launch_prob(sv_state *s, uint64_t mask, uint64_t value, double *part, double *out) {
    const int nm = __builtin_popcountll(mask);
    const uint64_t count = uint64_t(1) << (s->n - nm);
    uint64_t chunk;
    int blocks;
    red_geometry(count, &chunk, &blocks);
    const BitSpec spec = svi_bits_of(mask);
    if (s->dtype == SV_C128)
        hipLaunchKernelGGL((k_prob1<c128>), dim3(blocks), dim3(SVI_RED_THREADS), 0, s->stream,
                           static_cast<const c128 *>(s->d), count, chunk, spec, value, part);
    else
        hipLaunchKernelGGL((k_prob1<c64>), dim3(blocks), dim3(SVI_RED_THREADS), 0, s->stream,
                           static_cast<const c64 *>(s->d), count, chunk, spec, value, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_red2<1>), dim3(1), dim3(SVI_RED_THREADS), 0, s->stream, part, blocks, out);
    return hipGetLastError();
}

hipError_t svi_launch_collapse(sv_state *s, uint64_t mask, uint64_t value, double scale) {
    const uint64_t count = uint64_t(1) << s->n;
    const uint64_t nvb = (count + 255) / 256;
    const dim3 grid(unsigned(std::min<uint64_t>(nvb, uint64_t(1) << 20)));
    if (s->dtype == SV_C128)
        hipLaunchKernelGGL((k_collapse<c128>), grid, dim3(256), 0, s->stream, static_cast<c128 *>(s->d), count, mask,
                           value, scale, nvb);
    else
        hipLaunchKernelGGL((k_collapse<c64>), grid, dim3(256), 0, s->stream, static_cast<c64 *>(s->d), count, mask,
                           value, float(scale), nvb);
    return hipGetLastError();
}

// Sums of |alpha_j|^2 over nch consecutive chunks of `chunk` amplitudes
// starting at index lo (the same per-block walk and tree as the reductions).
hipError_t svi_launch_chunk_sums(sv_state *s, uint64_t lo, uint64_t chunk, int nch, double *part) {
    BitSpec none;
    none.count = 0;
    const uint64_t count = chunk * uint64_t(nch);
    if (s->dtype == SV_C128)
        hipLaunchKernelGGL((k_prob1<c128>), dim3(nch), dim3(SVI_RED_THREADS), 0, s->stream,
                           static_cast<const c128 *>(s->d) + lo, count, chunk, none, uint64_t(0), part);
    else
        hipLaunchKernelGGL((k_prob1<c64>), dim3(nch), dim3(SVI_RED_THREADS), 0, s->stream,
                           static_cast<const c64 *>(s->d) + lo, count, chunk, none, uint64_t(0), part);
    return hipGetLastError();
}

hipError_t svi_launch_inner(const sv_state *a, const sv_state *b, hipStream_t st, double *part, double *out) {
    const uint64_t count = uint64_t(1) << a->n;
    uint64_t chunk;
    int blocks;
    red_geometry(count, &chunk, &blocks);
    const dim3 g(blocks), t(SVI_RED_THREADS);
    if (a->dtype == SV_C128 && b->dtype == SV_C128)
        hipLaunchKernelGGL((k_inner1<c128, c128>), g, t, 0, st, static_cast<const c128 *>(a->d),
                           static_cast<const c128 *>(b->d), count, chunk, part);
    else if (a->dtype == SV_C128)
        hipLaunchKernelGGL((k_inner1<c128, c64>), g, t, 0, st, static_cast<const c128 *>(a->d),
                           static_cast<const c64 *>(b->d), count, chunk, part);
    else if (b->dtype == SV_C128)
        hipLaunchKernelGGL((k_inner1<c64, c128>), g, t, 0, st, static_cast<const c64 *>(a->d),
                           static_cast<const c128 *>(b->d), count, chunk, part);
    else
        hipLaunchKernelGGL((k_inner1<c64, c64>), g, t, 0, st, static_cast<const c64 *>(a->d),
                           static_cast<const c64 *>(b->d), count, chunk, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_red2<2>), dim3(1), dim3(SVI_RED_THREADS), 0, st, part, blocks, out);
    return hipGetLastError();
}
