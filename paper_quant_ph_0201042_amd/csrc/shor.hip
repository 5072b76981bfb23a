// Shor's factoring algorithm as sec. 5.1 runs it for 14-15-bit N: the
// modular exponentiation is computed classically, the QFT and the
// measurement run on the register, and steps 4-5 (continued fractions,
// order tests, gcd) plus the four improvements of sec. 5.1 run on the host.
//
// Register after step 3(c) with first-register outcome v: the equal
// superposition of every a in [0, 2^m) with x^a mod N = v.  The value
// x^a mod N is split as x^(ah 2^h) x^al with a = ah 2^h + al; both factors
// come from tables of 2^h and 2^(m-h) residues built on the device, so each
// amplitude costs one product and one remainder.  One pass counts the
// matches (nothing but the tables is read), a second writes the register
// (one HBM write of 2^m amplitudes).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "device_common.h"

using namespace svd;

namespace {

constexpr int kShorBlocks = 1024;
constexpr int kShorThreads = 256;

__host__ __device__ inline uint64_t mulmod(uint64_t a, uint64_t b, uint64_t N) {
    return (a * b) % N;  // a, b < N < 2^32
}

__host__ __device__ inline uint64_t powmod(uint64_t x, uint64_t e, uint64_t N) {
    uint64_t r = 1 % N, b = x % N;
    for (; e; e >>= 1) {
        if (e & 1) r = mulmod(r, b, N);
        b = mulmod(b, b, N);
    }
    return r;
}

// lo[i] = x^i mod N (i < 2^h), hi[i] = x^(i 2^h) mod N (i < 2^(m-h)).
__global__ void k_shor_tables(uint32_t *lo, uint32_t *hi, int h, int mh, uint64_t x, uint64_t N) {
    const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < (uint64_t(1) << h)) lo[i] = uint32_t(powmod(x, i, N));
    if (i < (uint64_t(1) << mh)) hi[i] = uint32_t(powmod(x, i << h, N));
}

__device__ __forceinline__ bool shor_match(uint64_t a, const uint32_t *lo, const uint32_t *hi, int h, uint64_t N,
                                           uint32_t v) {
    const uint64_t lmask = (uint64_t(1) << h) - 1;
    return mulmod(hi[a >> h], lo[a & lmask], N) == v;
}

// Per-block match counts (fixed grid, so the host sums kShorBlocks values).
__global__ __launch_bounds__(kShorThreads) void k_shor_count(const uint32_t *lo, const uint32_t *hi, int h,
                                                             uint64_t M, uint64_t N, uint32_t v,
                                                             unsigned long long *counts) {
    __shared__ unsigned long long part[kShorThreads / 64];
    unsigned long long c = 0;
    for (uint64_t a = uint64_t(blockIdx.x) * kShorThreads + threadIdx.x; a < M; a += uint64_t(gridDim.x) * kShorThreads)
        c += shor_match(a, lo, hi, h, N, v) ? 1 : 0;
    for (int o = 32; o; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kShorThreads / 64; ++w) t += part[w];
        counts[blockIdx.x] = t;
    }
}

template <typename T>
__global__ __launch_bounds__(kShorThreads) void k_shor_write(T *__restrict__ a, const uint32_t *lo,
                                                             const uint32_t *hi, int h, uint64_t M, uint64_t N,
                                                             uint32_t v, typename RealOf<T>::type amp) {
    using R = typename RealOf<T>::type;
    for (uint64_t j = uint64_t(blockIdx.x) * kShorThreads + threadIdx.x; j < M; j += uint64_t(gridDim.x) * kShorThreads) {
        T z;
        z.x = shor_match(j, lo, hi, h, N, v) ? amp : R(0);
        z.y = R(0);
        stnt(z, a + j);
    }
}

int sync(hipStream_t st) {
    hipError_t e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipGetLastError();
    return e == hipSuccess ? SV_OK : svi_fail("shor: synchronize", e);
}

unsigned bitlen(uint64_t v) {
    unsigned b = 0;
    for (; v; v >>= 1) ++b;
    return b;
}

uint64_t gcd64(uint64_t a, uint64_t b) {
    while (b) {
        const uint64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// ------------------------------------------------------------ steps 4-5 ---
// Step 4: the coprime k/r, 0 < k < r < N, with |y/2^m - k/r| <= 2^-(m+1),
// searched among the continued-fraction convergents of y/2^m (Legendre: a
// fraction that close is one; 2^m >= N^2 makes it unique).  The bound is
// tested exactly, as 2 |y r - k 2^m| <= r, in 128-bit integers.
uint64_t order_candidate(uint64_t y, int m, uint64_t N) {
    typedef unsigned __int128 u128;
    const u128 M = u128(1) << m;
    u128 num = y, den = M;
    u128 hp = 0, h = 1, kp = 1, k = 0;  // convergents h/k, previous hp/kp
    uint64_t found = 0;
    while (den != 0) {
        const u128 q = num / den;
        const u128 rem = num - q * den;
        num = den;
        den = rem;
        const u128 hn = q * h + hp, kn = q * k + kp;
        hp = h;
        h = hn;
        kp = k;
        k = kn;
        if (k >= N) break;
        if (h > 0 && h < k) {
            const u128 yk = u128(y) * k, hM = h * M;
            const u128 diff = yk > hM ? yk - hM : hM - yk;
            if (2 * diff <= k) found = uint64_t(k);
        }
    }
    return found;
}

// x^(r/2) -+ 1 against N; returns a nontrivial factor or 0.
uint64_t half_power_gcd(uint64_t N, uint64_t x, uint64_t r) {
    if (r == 0 || (r & 1)) return 0;
    const uint64_t hpow = powmod(x, r / 2, N);
    const uint64_t d1 = gcd64(N, (hpow + N - 1) % N), d2 = gcd64(N, (hpow + 1) % N);
    if (d1 > 1 && d1 < N) return d1;
    if (d2 > 1 && d2 < N) return d2;
    return 0;
}

// The failure tests of step 4 (x^r != 1, r odd, x^(r/2) = +-1) and step 5.
uint64_t plain_test(uint64_t N, uint64_t x, uint64_t r) {
    if (r == 0 || (r & 1) || powmod(x, r, N) != 1 % N) return 0;
    const uint64_t hpow = powmod(x, r / 2, N);
    if (hpow == 1 || hpow == N - 1) return 0;
    return half_power_gcd(N, x, r);
}

void classical(uint64_t N, uint64_t x, uint64_t y, int m, int improved, uint64_t r_prev, sv_shor_outcome *o) {
    std::memset(o, 0, sizeof *o);
    o->stage = SV_SHOR_FAIL;
    uint64_t r = order_candidate(y, m, N);
    int stage = SV_SHOR_PLAIN;
    if (r == 0 && improved) {
        const int64_t step[4] = {1, -1, 2, -2};
        for (int i = 0; i < 4 && r == 0; ++i) {
            const int64_t yy = int64_t(y) + step[i];
            if (yy >= 0 && uint64_t(yy) < (uint64_t(1) << m)) r = order_candidate(uint64_t(yy), m, N);
        }
        ++o->checks[0][r ? 0 : 1];
        stage = SV_SHOR_NEIGHBOR;
    }
    if (r == 0) return;
    o->r = r;
    if (!improved || powmod(x, r, N) == 1 % N) {
        const uint64_t f = plain_test(N, x, r);
        if (f) {
            o->factor = f;
            o->stage = stage;
        }
        return;
    }
    if ((r & 1) == 0) {  // GCD check although x^r != 1
        const uint64_t f = half_power_gcd(N, x, r);
        ++o->checks[1][f ? 0 : 1];
        if (f) {
            o->factor = f;
            o->stage = SV_SHOR_GCD;
            return;
        }
    }
    uint64_t f = 0;  // small factor check: the first multiple c r < N with x^(c r) = 1
    for (uint64_t c = 2; c * r < N; ++c)
        if (powmod(x, c * r, N) == 1 % N) {
            f = plain_test(N, x, c * r);
            break;
        }
    ++o->checks[2][f ? 0 : 1];
    if (f) {
        o->factor = f;
        o->stage = SV_SHOR_SMALL;
        return;
    }
    if (r_prev && r_prev != r) {  // LCM check with the previous candidate
        const uint64_t L = r_prev / gcd64(r_prev, r) * r;
        f = plain_test(N, x, L);
        ++o->checks[3][f ? 0 : 1];
        if (f) {
            o->factor = f;
            o->stage = SV_SHOR_LCM;
        }
    }
}

bool n_ok(uint64_t N) { return N >= 2 && N < (uint64_t(1) << 32); }

}  // namespace

extern "C" int sv_shor_prepare(sv_state *s, uint64_t N, uint64_t x, uint64_t a_star, uint64_t *count) {
    if (!s || !n_ok(N)) return SV_EINVAL;
    const int m = s->n;
    const uint64_t M = uint64_t(1) << m;
    if (a_star >= M) return SV_EINVAL;
    const int h = (m + 1) / 2, mh = m - h;
    const uint64_t xr = x % N;
    const uint32_t v = uint32_t(powmod(xr, a_star, N));
    const size_t nlo = size_t(1) << h, nhi = size_t(1) << mh;
    // scratch kept by the state: block counts, then the two residue tables
    const size_t bytes = (nlo + nhi) * sizeof(uint32_t) + kShorBlocks * sizeof(unsigned long long);
    hipError_t e = hipSuccess;
    if (bytes > s->work_cap) {
        if (s->work) {
            e = hipStreamSynchronize(s->stream);  // earlier calls' kernels may still read it
            if (e == hipSuccess) e = hipFree(s->work);
            s->work = nullptr;
            s->work_cap = 0;
            if (e != hipSuccess) return svi_fail("sv_shor_prepare: scratch", e);
        }
        e = hipMalloc(&s->work, bytes);
        if (e != hipSuccess) {
            s->work = nullptr;
            return svi_fail("sv_shor_prepare: scratch", e);
        }
        s->work_cap = bytes;
    }
    unsigned long long *d_counts = static_cast<unsigned long long *>(s->work);
    uint32_t *lo = reinterpret_cast<uint32_t *>(d_counts + kShorBlocks);
    uint32_t *hi = lo + nlo;
    std::vector<unsigned long long> counts(kShorBlocks);
    const unsigned tb = unsigned((std::max(nlo, nhi) + 255) / 256);
    hipLaunchKernelGGL(k_shor_tables, dim3(tb), dim3(256), 0, s->stream, lo, hi, h, mh, xr, N);
    e = hipGetLastError();
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_shor_count, dim3(kShorBlocks), dim3(kShorThreads), 0, s->stream, lo, hi, h, M, N, v,
                           d_counts);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(counts.data(), d_counts, kShorBlocks * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                           s->stream);
    int rc = e == hipSuccess ? sync(s->stream) : svi_fail("sv_shor_prepare: launch", e);
    uint64_t c = 0;
    for (unsigned long long b : counts) c += b;
    if (rc == SV_OK) {
        // c >= 1: a_star itself matches
        const double amp = 1.0 / std::sqrt(double(c));
        const uint64_t nvb = (M + kShorThreads - 1) / kShorThreads;
        const dim3 grid(unsigned(std::min<uint64_t>(nvb, uint64_t(1) << 16)));
        if (s->dtype == SV_C128)
            hipLaunchKernelGGL((k_shor_write<c128>), grid, dim3(kShorThreads), 0, s->stream,
                               static_cast<c128 *>(s->d), lo, hi, h, M, N, v, amp);
        else
            hipLaunchKernelGGL((k_shor_write<c64>), grid, dim3(kShorThreads), 0, s->stream, static_cast<c64 *>(s->d),
                               lo, hi, h, M, N, v, float(amp));
        e = hipGetLastError();
        rc = e == hipSuccess ? sync(s->stream) : svi_fail("sv_shor_prepare: launch", e);
    }
    if (rc == SV_OK && count) *count = c;
    return rc;
}

extern "C" int sv_shor_classical(uint64_t N, uint64_t x, uint64_t y, int m, int flags, uint64_t r_prev,
                                 sv_shor_outcome *out) {
    if (!out || !n_ok(N) || m < 1 || m > 62 || (flags & ~SV_SHOR_IMPROVED)) return SV_EINVAL;
    if (y >> m) return SV_EINVAL;
    classical(N, x % N, y, m, flags & SV_SHOR_IMPROVED, r_prev, out);
    return SV_OK;
}

extern "C" int sv_shor_factor(sv_state *s, uint64_t N, const uint64_t *x, const uint64_t *a_star, const double *u,
                              int64_t max_iters, int flags, uint64_t *y_out, sv_shor_result *res) {
    if (!s || !res || !n_ok(N) || max_iters < 0 || (max_iters > 0 && (!x || !a_star || !u))) return SV_EINVAL;
    if ((flags & ~SV_SHOR_IMPROVED) || s->n != int(2 * bitlen(N))) return SV_EINVAL;
    const int m = s->n;
    for (int64_t i = 0; i < max_iters; ++i)  // every draw is checked before any device work
        if (x[i] < 1 || x[i] >= N || (a_star[i] >> m) || !(u[i] >= 0.0 && u[i] < 1.0)) return SV_EINVAL;
    std::memset(res, 0, sizeof *res);
    res->stage = SV_SHOR_FAIL;
    uint64_t r_prev = 0;
    for (int64_t i = 0; i < max_iters; ++i) {
        if (y_out) y_out[i] = ~uint64_t(0);
        const uint64_t d = gcd64(x[i], N);  // step 2
        if (d > 1) {
            res->iterations = i + 1;
            res->factor = d;
            res->stage = SV_SHOR_GCDX;
            return SV_OK;
        }
        int rc = sv_shor_prepare(s, N, x[i], a_star[i], nullptr);
        if (rc == SV_OK) rc = sv_qft(s, 0, m, SV_QFT_BITREV);
        uint64_t j = 0;
        if (rc == SV_OK) rc = sv_measure(s, u[i], &j);
        if (rc != SV_OK) return rc;
        uint64_t y = 0;
        for (int b = 0; b < m; ++b) y |= ((j >> b) & 1) << (m - 1 - b);
        if (y_out) y_out[i] = y;
        sv_shor_outcome o;
        classical(N, x[i], y, m, flags & SV_SHOR_IMPROVED, r_prev, &o);
        for (int c = 0; c < 4; ++c) {
            res->checks[c][0] += o.checks[c][0];
            res->checks[c][1] += o.checks[c][1];
        }
        if (o.r) r_prev = o.r;
        if (o.factor) {
            res->iterations = i + 1;
            res->factor = o.factor;
            res->stage = o.stage;
            return SV_OK;
        }
    }
    return SV_OK;
}
