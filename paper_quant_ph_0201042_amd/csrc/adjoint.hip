// Adjoint (reverse-mode) gradient of an overlap loss, uncomputing the
// circuit in place instead of storing intermediate states.
//
// For psi_L = U_L ... U_1 psi_0, A = <phi|psi_L> and loss = 1 - |A|^2, the
// derivative with respect to an angle deviation eps_g of gate g is
//   dloss/deps_g = -2 Re(conj(A) <lambda_g| dU_g |psi_{g-1}>),
//   lambda_g = U_{g+1}^dagger ... U_L^dagger phi,
// (chain rule on the gate list).  The sweep walks g = L..1 keeping only psi
// and lambda: psi <- U_g^dagger psi (now psi_{g-1}), partial_g =
// <lambda| dU_g |psi>, lambda <- U_g^dagger lambda.  A gate's controls are
// exact, so dU_g has zero rows where a control bit is 0 (sec. 2.2.2 rows
// CTX[j] = I[j] do not depend on the angle) and only the control-1 subspace
// is visited.  For a parameterised gate one kernel reads both pairs, writes
// both updated pairs and accumulates the partial in FP64; other gates apply
// U^dagger to both states with the per-gate kernels.
#include <cstring>
#include <vector>

#include "device_common.h"

using namespace svd;

namespace {

constexpr int kAdjThreads = 256;
constexpr int kAdjBlocks = 1024;  // fixed grid: deterministic partial sums

template <typename R>
struct Mat2x {
    R v[8];  // U^dagger
    R d[8];  // dU
};

template <int W>
__device__ __forceinline__ void tree2(double (&x)[W], double *sh) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int w = 0; w < W; ++w) sh[w * kAdjThreads + tid] = x[w];
    __syncthreads();
    for (int st = kAdjThreads / 2; st > 0; st >>= 1) {
        if (tid < st) {
#pragma unroll
            for (int w = 0; w < W; ++w) sh[w * kAdjThreads + tid] += sh[w * kAdjThreads + tid + st];
        }
        __syncthreads();
    }
#pragma unroll
    for (int w = 0; w < W; ++w) x[w] = sh[w * kAdjThreads];
}

// One parameterised gate: pairs (i0, i0 | 2^b) over the control-1 subspace
// (zero bits inserted at spec, then ctrl set).  DIAG: the gate and its
// derivative are diagonal, so only the halves flagged in s0/s1 are read and
// written.  part[blockIdx.x] receives the block's FP64 partial
// sum of conj(lambda) . dU psi'.
template <typename T, bool DIAG>
__global__ __launch_bounds__(kAdjThreads) void k_adj_gate(T *__restrict__ psi, T *__restrict__ lam, uint64_t count,
                                                          int b, uint64_t ctrl, BitSpec spec,
                                                          Mat2x<typename RealOf<T>::type> m, int s0, int s1,
                                                          double *__restrict__ part) {
    using R = typename RealOf<T>::type;
    __shared__ double sh[2 * kAdjThreads];
    const uint64_t tb = uint64_t(1) << b;
    double acc_re = 0.0, acc_im = 0.0;
    const uint64_t stride = uint64_t(gridDim.x) * kAdjThreads;
    for (uint64_t t = uint64_t(blockIdx.x) * kAdjThreads + threadIdx.x; t < count; t += stride) {
        const uint64_t i0 = insert_zeros(t, spec) | ctrl;
        const uint64_t i1 = i0 | tb;
        if (DIAG) {
            // psi' = conj-diag * psi, d = diag(D) * psi'
            if (s0) {
                const T x = psi[i0], l = lam[i0];
                const T xn = cscale<T, R>(m.v[0], m.v[1], x);
                const T d = cscale<T, R>(m.d[0], m.d[1], xn);
                acc_re += double(l.x) * double(d.x) + double(l.y) * double(d.y);
                acc_im += double(l.x) * double(d.y) - double(l.y) * double(d.x);
                psi[i0] = xn;
                lam[i0] = cscale<T, R>(m.v[0], m.v[1], l);
            }
            if (s1) {
                const T y = psi[i1], l = lam[i1];
                const T yn = cscale<T, R>(m.v[6], m.v[7], y);
                const T d = cscale<T, R>(m.d[6], m.d[7], yn);
                acc_re += double(l.x) * double(d.x) + double(l.y) * double(d.y);
                acc_im += double(l.x) * double(d.y) - double(l.y) * double(d.x);
                psi[i1] = yn;
                lam[i1] = cscale<T, R>(m.v[6], m.v[7], l);
            }
        } else {
            const T x = psi[i0], y = psi[i1];
            const T lx = lam[i0], ly = lam[i1];
            const T xn = mac2<T, R>(m.v, 0, x, y);
            const T yn = mac2<T, R>(m.v, 4, x, y);
            const T d0 = mac2<T, R>(m.d, 0, xn, yn);
            const T d1 = mac2<T, R>(m.d, 4, xn, yn);
            acc_re += double(lx.x) * double(d0.x) + double(lx.y) * double(d0.y);
            acc_im += double(lx.x) * double(d0.y) - double(lx.y) * double(d0.x);
            acc_re += double(ly.x) * double(d1.x) + double(ly.y) * double(d1.y);
            acc_im += double(ly.x) * double(d1.y) - double(ly.y) * double(d1.x);
            psi[i0] = xn;
            psi[i1] = yn;
            lam[i0] = mac2<T, R>(m.v, 0, lx, ly);
            lam[i1] = mac2<T, R>(m.v, 4, lx, ly);
        }
    }
    double v2[2] = {acc_re, acc_im};
    tree2<2>(v2, sh);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = v2[0];
        part[2 * blockIdx.x + 1] = v2[1];
    }
}

// grad[g] = -2 Re(conj(A) p_g), p_g the sum of the gate's block partials in
// a fixed tree order; gates without a parameter get 0.
__global__ __launch_bounds__(kAdjThreads) void k_adj_finish(const double *__restrict__ part,
                                                            const int32_t *__restrict__ nblocks,
                                                            const double *__restrict__ A, double *__restrict__ grad) {
    __shared__ double sh[2 * kAdjThreads];
    const int g = blockIdx.x;
    const int nb = nblocks[g];
    const double *p = part + size_t(g) * 2 * kAdjBlocks;
    double v[2] = {0.0, 0.0};
    for (int k = threadIdx.x; k < nb; k += kAdjThreads) {
        v[0] += p[2 * k];
        v[1] += p[2 * k + 1];
    }
    tree2<2>(v, sh);
    if (threadIdx.x == 0) grad[g] = nb > 0 ? -2.0 * (A[0] * v[0] + A[1] * v[1]) : 0.0;
}

void dagger(const double U[8], double V[8]) {
    // V = U^dagger: v11 = conj(u11), v12 = conj(u21), v21 = conj(u12), v22 = conj(u22)
    V[0] = U[0];
    V[1] = -U[1];
    V[2] = U[4];
    V[3] = -U[5];
    V[4] = U[2];
    V[5] = -U[3];
    V[6] = U[6];
    V[7] = -U[7];
}

template <typename R>
Mat2x<R> to_mat2x(const double V[8], const double D[8]) {
    Mat2x<R> m;
    for (int i = 0; i < 8; ++i) {
        m.v[i] = R(V[i]);
        m.d[i] = R(D[i]);
    }
    return m;
}

template <typename T>
hipError_t launch_adj_gate(sv_state *psi, sv_state *lam, const PreparedGate &g, const double V[8],
                           const double D[8], double *part, int *nblocks_out) {
    using R = typename RealOf<T>::type;
    const int n = psi->n;
    const int b = n - 1 - g.q;
    const int nc = __builtin_popcountll(g.ctrl);
    const uint64_t count = (uint64_t(1) << n) >> (nc + 1);
    const BitSpec spec = svi_bits_of(g.ctrl | (uint64_t(1) << b));
    const int blocks = int(std::min<uint64_t>(kAdjBlocks, (count + kAdjThreads - 1) / kAdjThreads));
    *nblocks_out = blocks;
    const Mat2x<R> m = to_mat2x<R>(V, D);
    T *ps = static_cast<T *>(psi->d);
    T *la = static_cast<T *>(lam->d);
    const bool diag = V[2] == 0.0 && V[3] == 0.0 && V[4] == 0.0 && V[5] == 0.0 && D[2] == 0.0 && D[3] == 0.0 &&
                      D[4] == 0.0 && D[5] == 0.0;
    if (diag) {
        const int s0 = !(V[0] == 1.0 && V[1] == 0.0 && D[0] == 0.0 && D[1] == 0.0);
        const int s1 = !(V[6] == 1.0 && V[7] == 0.0 && D[6] == 0.0 && D[7] == 0.0);
        hipLaunchKernelGGL((k_adj_gate<T, true>), dim3(blocks), dim3(kAdjThreads), 0, psi->stream, ps, la, count, b,
                           g.ctrl, spec, m, s0, s1, part);
    } else {
        hipLaunchKernelGGL((k_adj_gate<T, false>), dim3(blocks), dim3(kAdjThreads), 0, psi->stream, ps, la, count, b,
                           g.ctrl, spec, m, 1, 1, part);
    }
    return hipGetLastError();
}

}  // namespace

struct AdjointBuffers {
    double *part = nullptr;    // ng * 2 * kAdjBlocks doubles
    int32_t *nblk = nullptr;   // ng
    double *grad = nullptr;    // ng
    double *A = nullptr;       // 2 (+ scratch partials for the inner product)
    double *red = nullptr;     // 2 * SVI_RED_BLOCKS + 8
    int32_t *h_nblk = nullptr; // pinned
    size_t cap = 0;            // gates
};

void svi_release_adjoint(sv_state *s) {
    if (!s->adj) return;
    AdjointBuffers *b = s->adj;
    (void)hipStreamSynchronize(s->stream);
    if (b->part) (void)hipFree(b->part);
    if (b->nblk) (void)hipFree(b->nblk);
    if (b->grad) (void)hipFree(b->grad);
    if (b->A) (void)hipFree(b->A);
    if (b->red) (void)hipFree(b->red);
    if (b->h_nblk) (void)hipHostFree(b->h_nblk);
    delete b;
    s->adj = nullptr;
}

namespace {
int ensure_adj(sv_state *s, size_t ng) {
    if (!s->adj) s->adj = new (std::nothrow) AdjointBuffers();
    if (!s->adj) return SV_ENOMEM;
    AdjointBuffers *b = s->adj;
    if (!b->A) {
        if (hipMalloc(reinterpret_cast<void **>(&b->A), 4 * sizeof(double)) != hipSuccess) return SV_ENOMEM;
        if (hipMalloc(reinterpret_cast<void **>(&b->red), (2 * SVI_RED_BLOCKS + 8) * sizeof(double)) != hipSuccess)
            return SV_ENOMEM;
    }
    if (ng > b->cap) {
        if (hipStreamSynchronize(s->stream) != hipSuccess) return SV_EDEVICE;
        if (b->part) (void)hipFree(b->part);
        if (b->nblk) (void)hipFree(b->nblk);
        if (b->grad) (void)hipFree(b->grad);
        if (b->h_nblk) (void)hipHostFree(b->h_nblk);
        b->part = nullptr;
        b->nblk = nullptr;
        b->grad = nullptr;
        b->h_nblk = nullptr;
        b->cap = 0;
        if (hipMalloc(reinterpret_cast<void **>(&b->part), ng * 2 * kAdjBlocks * sizeof(double)) != hipSuccess ||
            hipMalloc(reinterpret_cast<void **>(&b->nblk), ng * sizeof(int32_t)) != hipSuccess ||
            hipMalloc(reinterpret_cast<void **>(&b->grad), ng * sizeof(double)) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&b->h_nblk), ng * sizeof(int32_t), hipHostMallocDefault) !=
                hipSuccess)
            return SV_ENOMEM;
        b->cap = ng;
    }
    return SV_OK;
}
}  // namespace

extern "C" int sv_adjoint(sv_state *psi, sv_state *lam, const sv_gate *gates, int64_t ng, const int32_t *dparam,
                          double *grad, double a_out[2]) {
    if (!psi || !lam || ng < 0 || (ng > 0 && (!gates || !dparam || !grad))) return SV_EINVAL;
    if (psi->n != lam->n || psi->dtype != lam->dtype || psi == lam) return SV_EINVAL;
    std::vector<PreparedGate> prep;
    int rc = svi_prepare(psi->n, gates, ng, prep, nullptr);
    if (rc != SV_OK) return rc;
    std::vector<double> D(size_t(ng) * 8, 0.0);
    for (int64_t g = 0; g < ng; ++g) {
        const int w = dparam[g];
        if (w < 0) continue;
        if (w > 1 || gates[g].kind == SV_G_SWAP) return SV_EINVAL;
        if (svi_gate_dmatrix(&gates[g], w, &D[size_t(g) * 8]) != SV_OK) return SV_EINVAL;
    }
    if (ng == 0) {
        if (a_out) {
            double A[2];
            rc = sv_inner(lam, psi, A);
            if (rc != SV_OK) return rc;
            a_out[0] = A[0];
            a_out[1] = A[1];
        }
        return SV_OK;
    }
    rc = ensure_adj(psi, size_t(ng));
    if (rc != SV_OK) return rc;
    AdjointBuffers *B = psi->adj;
    // order lambda's pending work before psi's stream
    if (lam->stream != psi->stream) {
        hipEvent_t ev;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return SV_EDEVICE;
        hipError_t e = hipEventRecord(ev, lam->stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(psi->stream, ev, 0);
        (void)hipEventDestroy(ev);
        if (e != hipSuccess) return SV_EDEVICE;
    }
    // A = <phi|psi_L>
    hipError_t e = svi_launch_inner(lam, psi, psi->stream, B->red, B->A);
    if (e != hipSuccess) return svi_status_from_hip(e);

    // the reverse sweep runs on psi's stream for both states
    hipStream_t keep = lam->stream;
    lam->stream = psi->stream;
    for (int64_t g = ng - 1; g >= 0 && rc == SV_OK; --g) {
        const PreparedGate &p = prep[size_t(g)];
        int nb = 0;
        if (p.kind == SV_G_SWAP) {
            e = svi_launch_swap(psi, p.q, p.q2);
            if (e == hipSuccess) e = svi_launch_swap(lam, p.q, p.q2);
        } else {
            double V[8];
            dagger(p.U, V);
            if (dparam[g] < 0) {
                e = svi_launch_gate(psi, p.ctrl, p.q, V);
                if (e == hipSuccess) e = svi_launch_gate(lam, p.ctrl, p.q, V);
            } else {
                double *part = B->part + size_t(g) * 2 * kAdjBlocks;
                e = psi->dtype == SV_C128 ? launch_adj_gate<c128>(psi, lam, p, V, &D[size_t(g) * 8], part, &nb)
                                          : launch_adj_gate<c64>(psi, lam, p, V, &D[size_t(g) * 8], part, &nb);
            }
        }
        B->h_nblk[g] = nb;
        if (e != hipSuccess) rc = svi_status_from_hip(e);
    }
    lam->stream = keep;
    if (rc != SV_OK) return rc;
    if (hipMemcpyAsync(B->nblk, B->h_nblk, size_t(ng) * sizeof(int32_t), hipMemcpyHostToDevice, psi->stream) !=
        hipSuccess)
        return SV_EDEVICE;
    hipLaunchKernelGGL(k_adj_finish, dim3(unsigned(ng)), dim3(kAdjThreads), 0, psi->stream, B->part, B->nblk, B->A,
                       B->grad);
    if (hipGetLastError() != hipSuccess) return SV_EDEVICE;
    if (hipMemcpyAsync(grad, B->grad, size_t(ng) * sizeof(double), hipMemcpyDeviceToHost, psi->stream) != hipSuccess)
        return SV_EDEVICE;
    double A[2] = {0, 0};
    if (hipMemcpyAsync(A, B->A, 2 * sizeof(double), hipMemcpyDeviceToHost, psi->stream) != hipSuccess)
        return SV_EDEVICE;
    if (hipStreamSynchronize(psi->stream) != hipSuccess) return SV_EDEVICE;
    if (a_out) {
        a_out[0] = A[0];
        a_out[1] = A[1];
    }
    return SV_OK;
}
