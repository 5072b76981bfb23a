// Batched noisy trajectories: many independent registers evolved by the same
// gate list under the error model of sec. 3, each with its own random draws.
//
// Error model (sec. 3.1 depolarizing channel, sec. 3.2 operational error):
// every gate's angles get Gaussian deviations; after every gate each qubit it
// touches suffers sigma_x, sigma_y or sigma_z with probability p/3 each.  The
// draws of trajectory t for gate g come from a counter-based generator,
// Philox4x32-10 with key = seed and counter (t, g, slot, 0), so any
// trajectory can be recomputed alone (the CPU oracle reproduces them):
//   slot 0: u_i = (r_i + 0.5) 2^-32, rad = sqrt(-2 ln u0),
//           x = sigma rad cos(2 pi u1) (rotation angle),
//           y = sigma rad sin(2 pi u1) (phase angle);
//   touched qubit number i (ascending qubit order): slot 1 + i/2, words
//           2(i%2) (event iff r < floor(p 2^32)) and 2(i%2)+1 (type (3r)>>32:
//           sigma_x, sigma_y, sigma_z).
//
// Execution.  Between two multi-qubit gates, every qubit sees a run of
// one-qubit gates and Paulis; the run is folded into one 2x2 matrix per
// qubit and trajectory (composed in FP64, rounded once to the register
// precision).  Multi-qubit gates must be diagonal (controlled phases such
// as the C^{n-1}Z of the Grover iteration): they stay diagonal ops whose
// perturbed phase is also a per-trajectory matrix, and the Paulis that
// follow them open the next run.  A generator kernel fills the table of
// per-trajectory matrices; the run/diagonal program is then compiled by
// the fused-pass planner, and each pass is one launch over all trajectories
// (workgroup = trajectory x tile).  The whole launch sequence is captured in
// a HIP graph and replayed.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "device_common.h"
#include "fused.h"

using namespace svd;

namespace {

// ------------------------------------------------------------ device RNG

__host__ __device__ __forceinline__ uint32_t mulhi32(uint32_t a, uint32_t b) {
    return uint32_t((uint64_t(a) * uint64_t(b)) >> 32);
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies with the Weyl key schedule.  The host copy serves
// svb_trajectory_gates.
__host__ __device__ __forceinline__ void philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                                uint32_t k1, uint32_t (&o)[4]) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = mulhi32(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = mulhi32(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    o[0] = c0;
    o[1] = c1;
    o[2] = c2;
    o[3] = c3;
}

// ------------------------------------------------------------ descriptors

enum NFType : int32_t { NF_GATE = 0, NF_PAULI = 1 };

struct NFactor {
    int32_t type;     // NF_GATE or NF_PAULI
    int32_t kind;     // gate kind (NF_GATE)
    int32_t iarg;     // R_k exponent
    int32_t touched;  // NF_PAULI: rank of the qubit among the gate's touched qubits
    uint64_t gidx;    // index of the gate in the noisy sequence (Philox counter word 1)
    double p[8];      // base parameters of the gate
};

struct NSlot {
    int32_t first;  // factors [first, first + count), applied in order
    int32_t count;
};

struct NParams {
    uint64_t seed;
    uint64_t traj0;  // trajectory id of register 0
    double sigma;
    uint32_t pthresh;  // floor(p 2^32)
    uint32_t pad;
};

// ------------------------------------------------------------ device gate matrices

struct DC {
    double re, im;
};
__device__ __forceinline__ DC dmul(DC a, DC b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ DC dadd(DC a, DC b) { return {a.re + b.re, a.im + b.im}; }

struct DM {
    DC a, b, c, d;  // row-major 2x2
};
__device__ __forceinline__ DM mmul(const DM &x, const DM &y) {
    DM r;
    r.a = dadd(dmul(x.a, y.a), dmul(x.b, y.c));
    r.b = dadd(dmul(x.a, y.b), dmul(x.b, y.d));
    r.c = dadd(dmul(x.c, y.a), dmul(x.d, y.c));
    r.d = dadd(dmul(x.c, y.b), dmul(x.d, y.d));
    return r;
}

// U_R(theta) U_P1(phi) = [[c, -s e^{i phi}], [s, c e^{i phi}]]
__device__ __forceinline__ DM rot_phase(double theta, double phi) {
    double s, c, sp, cp;
    sincos(theta, &s, &c);
    sincos(phi, &sp, &cp);
    return DM{{c, 0.0}, {-s * cp, -s * sp}, {s, 0.0}, {c * cp, c * sp}};
}
__device__ __forceinline__ DM phase_shift(double phi) {
    double sp, cp;
    sincos(phi, &sp, &cp);
    return DM{{1.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {cp, sp}};
}

// Device twin of the host gate-matrix construction (same definitions as
// sv_gate_matrix; deviations already added to p).
__device__ DM gate_matrix(int kind, int iarg, const double *p) {
    const double kPi = 3.14159265358979323846;
    switch (kind) {
    case SV_G_H:
        if (p[0] == 0.0 && p[1] == 0.0) {
            const double h = 0.70710678118654757;  // sqrt(0.5), correctly rounded
            return DM{{h, 0}, {h, 0}, {h, 0}, {-h, 0}};
        }
        return rot_phase(kPi / 4 + p[0], kPi + p[1]);
    case SV_G_X:
        if (p[0] == 0.0 && p[1] == 0.0) return DM{{0, 0}, {1, 0}, {1, 0}, {0, 0}};
        return rot_phase(kPi / 2 + p[0], kPi + p[1]);
    case SV_G_Y: return DM{{0, 0}, {0, -1}, {0, 1}, {0, 0}};
    case SV_G_Z:
        if (p[1] == 0.0) return DM{{1, 0}, {0, 0}, {0, 0}, {-1, 0}};
        return phase_shift(kPi + p[1]);
    case SV_G_RK: return phase_shift(2.0 * kPi / ldexp(1.0, iarg) + p[1]);
    case SV_G_ROT: return rot_phase(p[0], p[1]);
    case SV_G_SU2: {
        const double r = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2] + p[3] * p[3]);
        const double a = p[0] / r, b = p[1] / r, c = p[2] / r, d = p[3] / r;
        return DM{{a, b}, {c, d}, {-c, d}, {a, -b}};
    }
    default:  // SV_G_U
        return DM{{p[0], p[1]}, {p[2], p[3]}, {p[4], p[5]}, {p[6], p[7]}};
    }
}

// One thread per (register, slot): the product of the slot's factors for
// that register's trajectory, rounded once to R.
template <typename R>
__global__ __launch_bounds__(256) void k_gen(const NFactor *__restrict__ fac, const NSlot *__restrict__ slots,
                                             uint32_t nslots, uint64_t nregs, const NParams *__restrict__ prm,
                                             R *__restrict__ table) {
    const uint64_t id = uint64_t(blockIdx.x) * 256 + threadIdx.x;
    if (id >= nregs * nslots) return;
    const uint64_t reg = id / nslots;
    const uint32_t sl = uint32_t(id - reg * nslots);
    const NParams P = *prm;
    const uint64_t traj = P.traj0 + reg;
    const uint32_t k0 = uint32_t(P.seed), k1 = uint32_t(P.seed >> 32);
    DM acc{{1, 0}, {0, 0}, {0, 0}, {1, 0}};
    const NSlot S = slots[sl];
    for (int f = 0; f < S.count; ++f) {
        const NFactor &F = fac[S.first + f];
        if (F.type == NF_GATE) {
            double p[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) p[i] = F.p[i];
            if (P.sigma != 0.0) {
                uint32_t r[4];
                philox(uint32_t(traj), uint32_t(F.gidx), 0u, 0u, k0, k1, r);
                const double u0 = (double(r[0]) + 0.5) * 0x1p-32;
                const double u1 = (double(r[1]) + 0.5) * 0x1p-32;
                const double rad = sqrt(-2.0 * log(u0));
                double s1, c1;
                sincos(2.0 * 3.14159265358979323846 * u1, &s1, &c1);
                const double x = P.sigma * rad * c1, y = P.sigma * rad * s1;
                if (F.kind == SV_G_H || F.kind == SV_G_X || F.kind == SV_G_ROT) {
                    p[0] += x;
                    p[1] += y;
                } else if (F.kind == SV_G_Z || F.kind == SV_G_RK) {
                    p[1] += y;
                }
            }
            acc = mmul(gate_matrix(F.kind, F.iarg, p), acc);
        } else {
            uint32_t r[4];
            philox(uint32_t(traj), uint32_t(F.gidx), 1u + uint32_t(F.touched / 2), 0u, k0, k1, r);
            const int w = 2 * (F.touched % 2);
            if (r[w] < P.pthresh) {
                const int t = int((uint64_t(r[w + 1]) * 3u) >> 32);
                const double zp[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                acc = mmul(gate_matrix(t == 0 ? SV_G_X : (t == 1 ? SV_G_Y : SV_G_Z), 0, zp), acc);
            }
        }
    }
    R *o = table + id * 8;
    o[0] = R(acc.a.re);
    o[1] = R(acc.a.im);
    o[2] = R(acc.b.re);
    o[3] = R(acc.b.im);
    o[4] = R(acc.c.re);
    o[5] = R(acc.c.im);
    o[6] = R(acc.d.re);
    o[7] = R(acc.d.im);
}

// Every register of the batch to |0...0>.  A dispatch holds at most 2^32
// work-items, so the grid walks virtual blocks vb < nvb.
template <typename T>
__global__ __launch_bounds__(256) void k_reset_batch(T *__restrict__ a, uint64_t total, int n, uint64_t nvb) {
    for (uint64_t vb = blockIdx.x; vb < nvb; vb += gridDim.x) {
        const uint64_t j = vb * 256 + threadIdx.x;
        if (j >= total) continue;
        T v;
        v.x = ((j & ((uint64_t(1) << n) - 1)) == 0) ? 1 : 0;
        v.y = 0;
        stnt(v, a + j);
    }
}

// Per register: |alpha_idx|^2 and the squared norm (FP64, fixed tree).
template <typename T>
__global__ __launch_bounds__(256) void k_result(const T *__restrict__ a, int n, uint64_t idx, double *__restrict__ out) {
    __shared__ double sh[256];
    const uint64_t reg = blockIdx.x;
    const T *r = a + (reg << n);
    const uint64_t N = uint64_t(1) << n;
    double acc = 0.0;
    for (uint64_t j = threadIdx.x; j < N; j += 256) {
        const T v = ldnt(r + j);
        acc += double(v.x) * double(v.x) + double(v.y) * double(v.y);
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (unsigned s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const T v = r[idx];
        out[2 * reg] = double(v.x) * double(v.x) + double(v.y) * double(v.y);
        out[2 * reg + 1] = sh[0];
    }
}

// Per register pair (one workgroup each): <a|b> (re, im), <a|a>, <b|b> in
// FP64 with a fixed tree, so a result depends only on n.
template <typename TA, typename TB>
__global__ __launch_bounds__(256) void k_pair_overlap(const TA *__restrict__ a, const TB *__restrict__ b, int n,
                                                      double *__restrict__ out) {
    __shared__ double sh[4][256];
    const uint64_t reg = blockIdx.x;
    const TA *ra = a + (reg << n);
    const TB *rb = b + (reg << n);
    const uint64_t N = uint64_t(1) << n;
    double re = 0.0, im = 0.0, aa = 0.0, bb = 0.0;
    for (uint64_t j = threadIdx.x; j < N; j += 256) {
        const TA u = ldnt(ra + j);
        const TB v = ldnt(rb + j);
        const double ux = double(u.x), uy = double(u.y), vx = double(v.x), vy = double(v.y);
        re += ux * vx + uy * vy;
        im += ux * vy - uy * vx;
        aa += ux * ux + uy * uy;
        bb += vx * vx + vy * vy;
    }
    sh[0][threadIdx.x] = re;
    sh[1][threadIdx.x] = im;
    sh[2][threadIdx.x] = aa;
    sh[3][threadIdx.x] = bb;
    __syncthreads();
    for (unsigned s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s)
            for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 4) out[4 * reg + threadIdx.x] = sh[threadIdx.x][0];
}

// Per register (one workgroup each): the measurement of sec. 2.2.3 with the
// draw r[reg].  Thread t sums its contiguous chunk of |alpha_j|^2 in index
// order; thread 0 walks the chunk sums, then the chosen chunk element by
// element: the smallest i whose running FP64 sum exceeds r; if r reaches
// the total, the last index of nonzero weight (0 for an all-zero register).
template <typename T>
__global__ __launch_bounds__(256) void k_measure_batch(const T *__restrict__ a, int n, const double *__restrict__ r,
                                                       uint64_t *__restrict__ index) {
    __shared__ double sh[256];
    const uint64_t reg = blockIdx.x;
    const T *ra = a + (reg << n);
    const uint64_t N = uint64_t(1) << n;
    const uint64_t chunk = N >= 256 ? N / 256 : 1;
    const uint64_t nch = N >= 256 ? 256 : N;
    double acc = 0.0;
    if (threadIdx.x < nch)
        for (uint64_t j = threadIdx.x * chunk; j < (threadIdx.x + 1) * chunk; ++j) {
            const T v = ra[j];
            acc += double(v.x) * double(v.x) + double(v.y) * double(v.y);
        }
    sh[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x != 0) return;
    const double rr = r[reg];
    auto w = [&](uint64_t j) {
        const T v = ra[j];
        return double(v.x) * double(v.x) + double(v.y) * double(v.y);
    };
    double cum = 0.0;
    int64_t last_nz = -1;
    for (uint64_t c = 0; c < nch; ++c) {
        if (sh[c] > 0.0) last_nz = int64_t(c);
        if (cum + sh[c] > rr) {
            double run = cum;
            int64_t last_in = -1;
            for (uint64_t j = c * chunk; j < (c + 1) * chunk; ++j) {
                const double wj = w(j);
                if (wj > 0.0) last_in = int64_t(j);
                run += wj;
                if (run > rr) {
                    index[reg] = j;
                    return;
                }
            }
            index[reg] = uint64_t(last_in < 0 ? 0 : last_in);  // rounding put r past the chunk
            return;
        }
        cum += sh[c];
    }
    uint64_t ans = 0;
    if (last_nz >= 0)
        for (uint64_t j = uint64_t(last_nz) * chunk; j < (uint64_t(last_nz) + 1) * chunk; ++j)
            if (w(j) > 0.0) ans = j;
    index[reg] = ans;
}

// ------------------------------------------------------------ host program

struct NoisyProgram {
    std::vector<NFactor> factors;
    std::vector<NSlot> slots;
    std::vector<PreparedGate> symbolic;  // one per slot, for the planner
};

bool is_one_qubit(const PreparedGate &g) { return g.kind != SV_G_SWAP && g.ctrl == 0; }

// Builds runs and diagonal ops from init + iters x iter (see the file
// comment).  Returns SV_ENOTSUP for a multi-qubit gate that is not diagonal
// or for a SWAP.
int build_program(int n, const std::vector<PreparedGate> &init, const std::vector<PreparedGate> &iter,
                  const sv_gate *init_rec, const sv_gate *iter_rec, int iters, bool pauli_on, uint32_t depol_kinds,
                  NoisyProgram &P) {
    std::vector<std::vector<NFactor>> run(static_cast<size_t>(n));
    auto emit_run = [&]() {
        for (int q = 0; q < n; ++q) {
            if (run[size_t(q)].empty()) continue;
            NSlot s;
            s.first = int32_t(P.factors.size());
            s.count = int32_t(run[size_t(q)].size());
            P.factors.insert(P.factors.end(), run[size_t(q)].begin(), run[size_t(q)].end());
            PreparedGate g{};
            g.kind = SV_G_U;
            g.q = q;
            g.q2 = -1;
            g.ctrl = 0;
            g.cls = GC_DENSE;
            g.slot = int32_t(P.slots.size());
            for (int i = 0; i < 8; ++i) g.U[i] = 0.0;
            P.slots.push_back(s);
            P.symbolic.push_back(g);
            run[size_t(q)].clear();
        }
    };
    uint64_t gidx = 0;
    auto add_gate = [&](const PreparedGate &g, const sv_gate &rec) -> int {
        NFactor f;
        std::memset(&f, 0, sizeof f);
        f.type = NF_GATE;
        f.kind = rec.kind;
        f.iarg = rec.iarg;
        f.gidx = gidx;
        for (int i = 0; i < 8; ++i) f.p[i] = rec.p[i];
        if (g.kind == SV_G_SWAP) return SV_ENOTSUP;
        const bool pauli = pauli_on && rec.kind >= 0 && rec.kind < 32 && ((depol_kinds >> rec.kind) & 1u);
        if (is_one_qubit(g)) {
            run[size_t(g.q)].push_back(f);
            if (pauli) {
                NFactor pf = f;
                pf.type = NF_PAULI;
                pf.touched = 0;
                run[size_t(g.q)].push_back(pf);
            }
        } else {
            if (g.cls != GC_DIAG) return SV_ENOTSUP;
            emit_run();
            NSlot s;
            s.first = int32_t(P.factors.size());
            s.count = 1;
            P.factors.push_back(f);
            PreparedGate d = g;
            d.slot = int32_t(P.slots.size());
            P.slots.push_back(s);
            P.symbolic.push_back(d);
            if (pauli) {
                // touched qubits in ascending qubit order (bit n-1-q)
                int i = 0;
                for (int q = 0; q < n; ++q) {
                    const uint64_t bit = uint64_t(1) << (n - 1 - q);
                    if (q != g.q && !(g.ctrl & bit)) continue;
                    NFactor pf = f;
                    pf.type = NF_PAULI;
                    pf.touched = i++;
                    run[size_t(q)].push_back(pf);
                }
            }
        }
        ++gidx;
        return SV_OK;
    };
    for (size_t i = 0; i < init.size(); ++i)
        if (int rc = add_gate(init[i], init_rec[i])) return rc;
    for (int it = 0; it < iters; ++it)
        for (size_t i = 0; i < iter.size(); ++i)
            if (int rc = add_gate(iter[i], iter_rec[i])) return rc;
    emit_run();
    return SV_OK;
}

uint32_t pauli_threshold(double p) {
    if (!(p > 0.0)) return 0;
    if (p >= 1.0) return 0xFFFFFFFFu;
    return uint32_t(std::floor(p * 4294967296.0));
}

}  // namespace

struct svb_batch {
    int n, B, dtype;
    void *d = nullptr;  // B registers of 2^n amplitudes, back to back
    hipStream_t user_stream = nullptr;
    hipStream_t stream = nullptr;  // private, capturable stream
    // program buffers (device)
    void *dfac = nullptr, *dslots = nullptr, *dpass = nullptr, *dops = nullptr, *dtable = nullptr;
    size_t cap_fac = 0, cap_slots = 0, cap_pass = 0, cap_ops = 0, cap_table = 0;
    NParams *dprm = nullptr;
    double *dres = nullptr, *hres = nullptr;  // 2 doubles per register
    double *dred = nullptr, *hred = nullptr;  // svb_fidelity / svb_measure: 4 words per register (lazy)
    int group = 0;                            // registers per pass launch (0 = all)
    int start = SVB_START_ZERO;               // reset the registers, or keep their contents
    uint32_t depol_kinds = 0xFFFFFFFFu;       // gate kinds followed by depolarizing draws
    hipGraphExec_t gexec = nullptr;
    uint64_t gkey = 0;  // signature of the captured program
    double last_ms = 0.0;
};

namespace {

int grow(void **p, size_t *cap, size_t bytes) {
    if (bytes <= *cap) return SV_OK;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    if (hipMalloc(p, bytes) != hipSuccess) return SV_ENOMEM;
    *cap = bytes;
    return SV_OK;
}

uint64_t fnv(const void *data, size_t len, uint64_t h) {
    const unsigned char *c = static_cast<const unsigned char *>(data);
    for (size_t i = 0; i < len; ++i) h = (h ^ c[i]) * 1099511628211ull;
    return h;
}

}  // namespace

extern "C" int svb_create(int n, int batch, int dtype, void *hip_stream, svb_batch **out) {
    if (!out) return SV_EINVAL;
    *out = nullptr;
    if (n < 1 || n > SV_MAX_QUBITS || batch < 1 || (dtype != SV_C64 && dtype != SV_C128)) return SV_EINVAL;
    svb_batch *b = new (std::nothrow) svb_batch();
    if (!b) return SV_ENOMEM;
    b->n = n;
    b->B = batch;
    b->dtype = dtype;
    b->user_stream = static_cast<hipStream_t>(hip_stream);
    const size_t bytes = (size_t(batch) << n) * size_t(dtype);
    if (hipMalloc(&b->d, bytes) != hipSuccess || hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&b->dprm), sizeof(NParams)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void **>(&b->dres), size_t(batch) * 2 * sizeof(double)) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&b->hres), size_t(batch) * 2 * sizeof(double),
                      hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        svb_destroy(b);
        return SV_ENOMEM;
    }
    *out = b;
    return SV_OK;
}

extern "C" int svb_destroy(svb_batch *b) {
    if (!b) return SV_OK;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    for (void *p : {b->d, b->dfac, b->dslots, b->dpass, b->dops, b->dtable, static_cast<void *>(b->dprm),
                    static_cast<void *>(b->dres), static_cast<void *>(b->dred)})
        if (p) (void)hipFree(p);
    if (b->hred) (void)hipHostFree(b->hred);
    if (b->hres) (void)hipHostFree(b->hres);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return SV_OK;
}

extern "C" int svb_info(const svb_batch *b, int *n, int *batch, int *dtype) {
    if (!b) return SV_EINVAL;
    if (n) *n = b->n;
    if (batch) *batch = b->B;
    if (dtype) *dtype = b->dtype;
    return SV_OK;
}

extern "C" int svb_get_group(const svb_batch *b, int *regs_per_launch) {
    if (!b || !regs_per_launch) return SV_EINVAL;
    *regs_per_launch = b->group;
    return SV_OK;
}

extern "C" int svb_state(svb_batch *b, int reg, void **dev_ptr) {
    if (!b || !dev_ptr || reg < 0 || reg >= b->B) return SV_EINVAL;
    *dev_ptr = static_cast<char *>(b->d) + ((size_t(reg) << b->n) * size_t(b->dtype));
    return SV_OK;
}

extern "C" int svb_set_start(svb_batch *b, int mode) {
    if (!b || (mode != SVB_START_ZERO && mode != SVB_START_KEEP)) return SV_EINVAL;
    b->start = mode;  // part of the captured graph's key
    return SV_OK;
}

extern "C" int svb_set_noise_kinds(svb_batch *b, uint32_t depolarize_kinds) {
    if (!b) return SV_EINVAL;
    b->depol_kinds = depolarize_kinds;  // changes the program, hence the graph key
    return SV_OK;
}

extern "C" int svb_set_group(svb_batch *b, int regs_per_launch) {
    if (!b || regs_per_launch < 0 || regs_per_launch > b->B) return SV_EINVAL;
    if (regs_per_launch != 0 && b->B % regs_per_launch != 0) return SV_EINVAL;
    if (b->group != regs_per_launch && b->gexec) {
        (void)hipGraphExecDestroy(b->gexec);
        b->gexec = nullptr;
        b->gkey = 0;
    }
    b->group = regs_per_launch;
    return SV_OK;
}

extern "C" int svb_plan(int n, int dtype, const sv_gate *init, int64_t n_init, const sv_gate *iter, int64_t n_iter,
                        int iters, int64_t *npasses, int64_t *nslots) {
    if (n < 1 || n > SV_MAX_QUBITS || (dtype != SV_C64 && dtype != SV_C128) || n_init < 0 || n_iter < 0 || iters < 0 ||
        (n_init > 0 && !init) || (n_iter > 0 && !iter) || !npasses || !nslots)
        return SV_EINVAL;
    std::vector<PreparedGate> pi, pt;
    int rc = svi_prepare(n, init, n_init, pi, nullptr);
    if (rc == SV_OK) rc = svi_prepare(n, iter, n_iter, pt, nullptr);
    if (rc != SV_OK) return rc;
    if (uint64_t(n_init) + uint64_t(iters) * uint64_t(n_iter) > 0xFFFFFFFFull) return SV_EINVAL;
    NoisyProgram prog;
    rc = build_program(n, pi, pt, init, iter, iters, true, 0xFFFFFFFFu, prog);
    if (rc != SV_OK) return rc;
    FusedProgram fp;
    rc = svi_fused_compile(n, dtype, prog.symbolic.data(), int64_t(prog.symbolic.size()), fp);
    if (rc != SV_OK) return rc;
    *npasses = int64_t(fp.passes.size());
    *nslots = int64_t(prog.slots.size());
    return SV_OK;
}

extern "C" int svb_jit_source(int n, int dtype, const sv_gate *init, int64_t n_init, const sv_gate *iter,
                              int64_t n_iter, int iters, int64_t pass, char *buf, int64_t cap, int64_t *len) {
    if (n < 1 || n > SV_MAX_QUBITS || (dtype != SV_C64 && dtype != SV_C128) || n_init < 0 || n_iter < 0 || iters < 0 ||
        (n_init > 0 && !init) || (n_iter > 0 && !iter) || !len || pass < 0)
        return SV_EINVAL;
    std::vector<PreparedGate> pi, pt;
    int rc = svi_prepare(n, init, n_init, pi, nullptr);
    if (rc == SV_OK) rc = svi_prepare(n, iter, n_iter, pt, nullptr);
    if (rc != SV_OK) return rc;
    if (uint64_t(n_init) + uint64_t(iters) * uint64_t(n_iter) > 0xFFFFFFFFull) return SV_EINVAL;
    NoisyProgram prog;
    rc = build_program(n, pi, pt, init, iter, iters, true, 0xFFFFFFFFu, prog);
    if (rc != SV_OK) return rc;
    FusedProgram fp;
    rc = svi_fused_compile(n, dtype, prog.symbolic.data(), int64_t(prog.symbolic.size()), fp);
    if (rc != SV_OK) return rc;
    fp.batched = true;
    if (pass >= int64_t(fp.passes.size())) return SV_EINVAL;
    const std::string s = svi_jit_pass_source(dtype, fp, size_t(pass));
    *len = int64_t(s.size());
    if (buf && cap > 0) {
        const size_t m = std::min<size_t>(s.size(), size_t(cap - 1));
        std::memcpy(buf, s.data(), m);
        buf[m] = '\0';
    }
    return SV_OK;
}

extern "C" int svb_run_noisy(svb_batch *b, const sv_gate *init, int64_t n_init, const sv_gate *iter, int64_t n_iter,
                             int iters, double sigma, double p, uint64_t seed, uint64_t traj_offset,
                             uint64_t target_index, double *prob, double *norm2) {
    if (!b || n_init < 0 || n_iter < 0 || iters < 0 || (n_init > 0 && !init) || (n_iter > 0 && !iter)) return SV_EINVAL;
    if (!(sigma >= 0.0) || !std::isfinite(sigma) || !(p >= 0.0) || p > 1.0) return SV_EINVAL;
    if (target_index >> b->n) return SV_EINVAL;
    if (traj_offset + uint64_t(b->B) - 1 > 0xFFFFFFFFull) return SV_EINVAL;  // counter word 0 is 32-bit
    const int n = b->n;
    std::vector<PreparedGate> pi, pt;
    int rc = svi_prepare(n, init, n_init, pi, nullptr);
    if (rc == SV_OK) rc = svi_prepare(n, iter, n_iter, pt, nullptr);
    if (rc != SV_OK) return rc;
    const uint64_t total_gates = uint64_t(n_init) + uint64_t(iters) * uint64_t(n_iter);
    if (total_gates > 0xFFFFFFFFull) return SV_EINVAL;  // counter word 1 is 32-bit
    NoisyProgram prog;
    rc = build_program(n, pi, pt, init, iter, iters, true, b->depol_kinds, prog);
    if (rc != SV_OK) return rc;
    FusedProgram fp;
    rc = svi_fused_compile(n, b->dtype, prog.symbolic.data(), int64_t(prog.symbolic.size()), fp);
    if (rc != SV_OK) return rc;
    fp.batched = true;
    const uint32_t nslots = uint32_t(prog.slots.size());
    const size_t rsz = b->dtype == SV_C128 ? sizeof(double) : sizeof(float);
    const size_t table_bytes = size_t(b->B) * nslots * 8 * rsz;

    // signature of everything the captured graph depends on
    uint64_t key = 1469598103934665603ull;
    key = fnv(prog.factors.data(), prog.factors.size() * sizeof(NFactor), key);
    key = fnv(prog.slots.data(), prog.slots.size() * sizeof(NSlot), key);
    key = fnv(fp.passes.data(), fp.passes.size() * sizeof(FPass), key);
    key = fnv(fp.ops.data(), fp.ops.size() * sizeof(FOp), key);
    key = fnv(&target_index, sizeof target_index, key);
    key = fnv(&b->group, sizeof b->group, key);
    key = fnv(&b->start, sizeof b->start, key);
    const int use_jit = svi_config().fused_jit;
    key = fnv(&use_jit, sizeof use_jit, key);
    // the specialised kernels also depend on the matrix-core and register settings
    const int use_mfma = svi_config().batch_mfma, waves = svi_config().batch_waves, cb = svi_config().batch_const_bits;
    key = fnv(&use_mfma, sizeof use_mfma, key);
    key = fnv(&waves, sizeof waves, key);
    key = fnv(&cb, sizeof cb, key);
    key = fnv(fp.generic.data(), fp.generic.size(), key);

    // order the caller's pending work before this run
    hipEvent_t ev;
    hipError_t he = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (he != hipSuccess) return svi_fail("svb_run_noisy: event create", he);
    he = hipEventRecord(ev, b->user_stream);
    if (he == hipSuccess) he = hipStreamWaitEvent(b->stream, ev, 0);
    if (he != hipSuccess) {
        (void)hipEventDestroy(ev);
        return svi_fail("svb_run_noisy: order after caller stream", he);
    }

    if (key != b->gkey || !b->gexec) {
        if (b->gexec) {
            (void)hipStreamSynchronize(b->stream);
            (void)hipGraphExecDestroy(b->gexec);
            b->gexec = nullptr;
            b->gkey = 0;
        }
        if (grow(&b->dfac, &b->cap_fac, std::max<size_t>(1, prog.factors.size()) * sizeof(NFactor)) ||
            grow(&b->dslots, &b->cap_slots, std::max<size_t>(1, prog.slots.size()) * sizeof(NSlot)) ||
            grow(&b->dpass, &b->cap_pass, std::max<size_t>(1, fp.passes.size()) * sizeof(FPass)) ||
            grow(&b->dops, &b->cap_ops, std::max<size_t>(1, fp.ops.size()) * sizeof(FOp)) ||
            grow(&b->dtable, &b->cap_table, std::max<size_t>(1, table_bytes))) {
            (void)hipEventDestroy(ev);
            return SV_ENOMEM;
        }
        // synchronous uploads (host vectors are temporaries)
        if ((!prog.factors.empty() && hipMemcpy(b->dfac, prog.factors.data(), prog.factors.size() * sizeof(NFactor),
                                                hipMemcpyHostToDevice) != hipSuccess) ||
            (!prog.slots.empty() &&
             hipMemcpy(b->dslots, prog.slots.data(), prog.slots.size() * sizeof(NSlot), hipMemcpyHostToDevice) !=
                 hipSuccess) ||
            (!fp.passes.empty() &&
             hipMemcpy(b->dpass, fp.passes.data(), fp.passes.size() * sizeof(FPass), hipMemcpyHostToDevice) !=
                 hipSuccess) ||
            (!fp.ops.empty() &&
             hipMemcpy(b->dops, fp.ops.data(), fp.ops.size() * sizeof(FOp), hipMemcpyHostToDevice) != hipSuccess)) {
            (void)hipEventDestroy(ev);
            return svi_fail("svb_run_noisy: program upload", hipErrorInvalidValue);
        }
        // specialised pass kernels are compiled and loaded before the capture
        std::vector<hipFunction_t> jit;
        if (use_jit) {
            int device = 0;
            if (hipGetDevice(&device) != hipSuccess) {
                (void)hipEventDestroy(ev);
                return SV_EDEVICE;
            }
            rc = svi_jit_prepare(device, b->dtype, fp, jit);
            if (rc != SV_OK) {
                (void)hipEventDestroy(ev);
                return rc;
            }
        }
        // capture: reset (unless the registers keep their contents), matrix
        // generation, passes, per-register results
        hipGraph_t graph;
        he = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
        if (he != hipSuccess) {
            (void)hipEventDestroy(ev);
            return svi_fail("svb_run_noisy: begin capture", he);
        }
        hipError_t e = hipSuccess;
        if (b->start == SVB_START_ZERO) {
            const uint64_t total = uint64_t(b->B) << n;
            const uint64_t rvb = (total + 255) / 256;
            const dim3 rgrid(unsigned(std::min<uint64_t>(rvb, uint64_t(1) << 20)));
            if (b->dtype == SV_C128)
                hipLaunchKernelGGL((k_reset_batch<c128>), rgrid, dim3(256), 0, b->stream, static_cast<c128 *>(b->d),
                                   total, n, rvb);
            else
                hipLaunchKernelGGL((k_reset_batch<c64>), rgrid, dim3(256), 0, b->stream, static_cast<c64 *>(b->d),
                                   total, n, rvb);
            e = hipGetLastError();
        }
        const uint64_t nthreads = uint64_t(b->B) * nslots;
        if (e == hipSuccess && nthreads > 0) {
            const dim3 ggrid(unsigned((nthreads + 255) / 256));
            if (b->dtype == SV_C128)
                hipLaunchKernelGGL((k_gen<double>), ggrid, dim3(256), 0, b->stream,
                                   static_cast<const NFactor *>(b->dfac), static_cast<const NSlot *>(b->dslots), nslots,
                                   uint64_t(b->B), b->dprm, static_cast<double *>(b->dtable));
            else
                hipLaunchKernelGGL((k_gen<float>), ggrid, dim3(256), 0, b->stream,
                                   static_cast<const NFactor *>(b->dfac), static_cast<const NSlot *>(b->dslots), nslots,
                                   uint64_t(b->B), b->dprm, static_cast<float *>(b->dtable));
            e = hipGetLastError();
        }
        const int group = b->group > 0 ? b->group : b->B;
        const size_t amp = size_t(b->dtype);
        for (int g0 = 0; g0 < b->B && e == hipSuccess; g0 += group) {
            FusedLaunch L;
            L.state = static_cast<char *>(b->d) + (size_t(g0) << n) * amp;
            L.n = n;
            L.dtype = b->dtype;
            L.stream = b->stream;
            L.table = static_cast<char *>(b->dtable) + size_t(g0) * nslots * 8 * rsz;
            L.nslots = nslots;
            L.nregs = uint64_t(group);
            for (const FusedProgram::Item &it : fp.items) {
                if (it.swap) {
                    e = hipErrorInvalidValue;  // programs have no swaps
                    break;
                }
                const int k = fp.passes[size_t(it.pass)].k;
                const FPass *dp = static_cast<const FPass *>(b->dpass) + it.pass;
                const FOp *dops = static_cast<const FOp *>(b->dops);
                e = (jit.empty() || !jit[size_t(it.pass)])
                        ? svi_fused_launch_pass(L, k, dp, dops)
                        : svi_jit_launch(jit[size_t(it.pass)], L, k, std::min(fp.m, k), dp, dops);
                if (e != hipSuccess) break;
            }
        }
        if (e == hipSuccess) {
            if (b->dtype == SV_C128)
                hipLaunchKernelGGL((k_result<c128>), dim3(unsigned(b->B)), dim3(256), 0, b->stream,
                                   static_cast<const c128 *>(b->d), n, target_index, b->dres);
            else
                hipLaunchKernelGGL((k_result<c64>), dim3(unsigned(b->B)), dim3(256), 0, b->stream,
                                   static_cast<const c64 *>(b->d), n, target_index, b->dres);
            e = hipGetLastError();
        }
        const hipError_t ec = hipStreamEndCapture(b->stream, &graph);
        if (e != hipSuccess || ec != hipSuccess) {
            if (ec == hipSuccess) (void)hipGraphDestroy(graph);
            (void)hipEventDestroy(ev);
            return svi_fail(e != hipSuccess ? "svb_run_noisy: launch during capture" : "svb_run_noisy: end capture",
                            e != hipSuccess ? e : ec);
        }
        const hipError_t ei = hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) {
            b->gexec = nullptr;
            (void)hipEventDestroy(ev);
            return svi_fail("svb_run_noisy: graph instantiate", ei);
        }
        b->gkey = key;
    }
    // run parameters live in device memory read by the generator, so the
    // captured graph is reused across seeds, sigma, p and trajectory ids
    NParams P;
    std::memset(&P, 0, sizeof P);
    P.seed = seed;
    P.traj0 = traj_offset;
    P.sigma = sigma;
    P.pthresh = pauli_threshold(p);
    he = hipMemcpyAsync(b->dprm, &P, sizeof P, hipMemcpyHostToDevice, b->stream);
    if (he != hipSuccess) {
        (void)hipEventDestroy(ev);
        return svi_fail("svb_run_noisy: parameter upload", he);
    }
    hipEvent_t t0, t1;
    (void)hipEventCreate(&t0);
    (void)hipEventCreate(&t1);
    (void)hipEventRecord(t0, b->stream);
    const char *stage = "graph launch";
    hipError_t e = hipGraphLaunch(b->gexec, b->stream);
    (void)hipEventRecord(t1, b->stream);
    if (e == hipSuccess) {
        stage = "result copy";
        e = hipMemcpyAsync(b->hres, b->dres, size_t(b->B) * 2 * sizeof(double), hipMemcpyDeviceToHost, b->stream);
    }
    if (e == hipSuccess) {
        stage = "synchronize";
        e = hipStreamSynchronize(b->stream);
    }
    float ms = 0.f;
    if (e == hipSuccess) (void)hipEventElapsedTime(&ms, t0, t1);
    b->last_ms = double(ms);
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    // later work on the caller's stream sees the results
    if (e == hipSuccess) e = hipEventRecord(ev, b->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->user_stream, ev, 0);
    (void)hipEventDestroy(ev);
    if (e != hipSuccess) return svi_fail(stage, e);
    for (int r = 0; r < b->B; ++r) {
        if (prob) prob[r] = b->hres[2 * r];
        if (norm2) norm2[r] = b->hres[2 * r + 1];
    }
    return SV_OK;
}

extern "C" int svb_last_run_ms(const svb_batch *b, double *ms) {
    if (!b || !ms) return SV_EINVAL;
    *ms = b->last_ms;
    return SV_OK;
}

// One trajectory of the error model as an explicit gate list, for the plain
// per-gate path: every gate with its drawn deviations added to its angles
// (same kinds, so sv_run builds the same matrices), followed by the Pauli
// gates its touched qubits drew.  Same draws as svb_run_noisy.
extern "C" int svb_trajectory_gates(int n, const sv_gate *init, int64_t n_init, const sv_gate *iter, int64_t n_iter,
                                    int iters, double sigma, double p, uint64_t seed, uint64_t traj,
                                    uint32_t depolarize_kinds, sv_gate *out, int64_t cap, int64_t *count) {
    if (!count || n < 1 || n > SV_MAX_QUBITS || n_init < 0 || n_iter < 0 || iters < 0 || cap < 0 ||
        (n_init > 0 && !init) || (n_iter > 0 && !iter) || (cap > 0 && !out))
        return SV_EINVAL;
    *count = 0;
    if (!(sigma >= 0.0) || !std::isfinite(sigma) || !(p >= 0.0) || p > 1.0 || traj > 0xFFFFFFFFull) return SV_EINVAL;
    std::vector<PreparedGate> chk;
    int rc = svi_prepare(n, init, n_init, chk, nullptr);
    if (rc == SV_OK) rc = svi_prepare(n, iter, n_iter, chk, nullptr);
    if (rc != SV_OK) return rc;
    for (int64_t i = 0; i < n_init; ++i)
        if (init[i].kind == SV_G_SWAP) return SV_ENOTSUP;
    for (int64_t i = 0; i < n_iter; ++i)
        if (iter[i].kind == SV_G_SWAP) return SV_ENOTSUP;
    const uint64_t total = uint64_t(n_init) + uint64_t(iters) * uint64_t(n_iter);
    if (total > 0xFFFFFFFFull) return SV_EINVAL;
    const uint32_t pt = pauli_threshold(p);
    const uint32_t k0 = uint32_t(seed), k1 = uint32_t(seed >> 32);
    const double kTwoPi = 6.283185307179586476925;
    int64_t w = 0;
    auto put = [&](const sv_gate &g) {
        if (w < cap) out[w] = g;
        ++w;
    };
    for (uint64_t gi = 0; gi < total; ++gi) {
        const sv_gate &src = gi < uint64_t(n_init) ? init[gi] : iter[(gi - uint64_t(n_init)) % uint64_t(n_iter)];
        sv_gate g = src;
        if (sigma != 0.0) {
            uint32_t r[4];
            philox(uint32_t(traj), uint32_t(gi), 0u, 0u, k0, k1, r);
            const double u0 = (double(r[0]) + 0.5) * 0x1p-32;
            const double u1 = (double(r[1]) + 0.5) * 0x1p-32;
            const double rad = std::sqrt(-2.0 * std::log(u0));
            const double x = sigma * rad * std::cos(kTwoPi * u1), y = sigma * rad * std::sin(kTwoPi * u1);
            if (g.kind == SV_G_H || g.kind == SV_G_X || g.kind == SV_G_ROT) {
                g.p[0] += x;
                g.p[1] += y;
            } else if (g.kind == SV_G_Z || g.kind == SV_G_RK) {
                g.p[1] += y;
            }
        }
        put(g);
        if (pt == 0 || !(src.kind >= 0 && src.kind < 32 && ((depolarize_kinds >> src.kind) & 1u))) continue;
        int i = 0;
        for (int q = 0; q < n; ++q) {
            const uint64_t bit = uint64_t(1) << (n - 1 - q);
            if (q != src.target && !(src.ctrl & bit)) continue;
            uint32_t r[4];
            philox(uint32_t(traj), uint32_t(gi), 1u + uint32_t(i / 2), 0u, k0, k1, r);
            const int wd = 2 * (i % 2);
            ++i;
            if (r[wd] >= pt) continue;
            const int t = int((uint64_t(r[wd + 1]) * 3u) >> 32);
            sv_gate pg;
            std::memset(&pg, 0, sizeof pg);
            pg.kind = t == 0 ? SV_G_X : (t == 1 ? SV_G_Y : SV_G_Z);
            pg.target = q;
            pg.target2 = -1;
            put(pg);
        }
    }
    *count = w;
    return SV_OK;
}

namespace {

int ensure_red(svb_batch *b) {
    if (b->dred) return SV_OK;
    const size_t bytes = size_t(b->B) * 4 * sizeof(double);
    if (hipMalloc(reinterpret_cast<void **>(&b->dred), bytes) != hipSuccess) {
        (void)hipGetLastError();
        b->dred = nullptr;
        return SV_ENOMEM;
    }
    if (hipHostMalloc(reinterpret_cast<void **>(&b->hred), bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(b->dred);
        b->dred = nullptr;
        b->hred = nullptr;
        return SV_ENOMEM;
    }
    return SV_OK;
}

}  // namespace

extern "C" int svb_fidelity(svb_batch *a, svb_batch *b, double *fid, double *overlap) {
    if (!a || !b || (!fid && !overlap) || a == b || a->n != b->n || a->B != b->B) return SV_EINVAL;
    if (int rc = ensure_red(a)) return rc;
    hipStream_t st = a->user_stream;
    hipEvent_t ev;
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) return svi_fail("svb_fidelity: event create", e);
    e = hipEventRecord(ev, b->user_stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, ev, 0);
    (void)hipEventDestroy(ev);
    if (e != hipSuccess) return svi_fail("svb_fidelity: order streams", e);
    const dim3 grid(unsigned(a->B)), blk(256);
    if (a->dtype == SV_C128 && b->dtype == SV_C128)
        hipLaunchKernelGGL((k_pair_overlap<c128, c128>), grid, blk, 0, st, static_cast<const c128 *>(a->d),
                           static_cast<const c128 *>(b->d), a->n, a->dred);
    else if (a->dtype == SV_C128)
        hipLaunchKernelGGL((k_pair_overlap<c128, c64>), grid, blk, 0, st, static_cast<const c128 *>(a->d),
                           static_cast<const c64 *>(b->d), a->n, a->dred);
    else if (b->dtype == SV_C128)
        hipLaunchKernelGGL((k_pair_overlap<c64, c128>), grid, blk, 0, st, static_cast<const c64 *>(a->d),
                           static_cast<const c128 *>(b->d), a->n, a->dred);
    else
        hipLaunchKernelGGL((k_pair_overlap<c64, c64>), grid, blk, 0, st, static_cast<const c64 *>(a->d),
                           static_cast<const c64 *>(b->d), a->n, a->dred);
    e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(a->hred, a->dred, size_t(a->B) * 4 * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return svi_fail("svb_fidelity", e);
    for (int r = 0; r < a->B; ++r) {
        const double *o = a->hred + 4 * r;
        if (overlap) {
            overlap[2 * r] = o[0];
            overlap[2 * r + 1] = o[1];
        }
        if (fid) fid[r] = (o[2] > 0.0 && o[3] > 0.0) ? (o[0] * o[0] + o[1] * o[1]) / (o[2] * o[3]) : 0.0;
    }
    return SV_OK;
}

extern "C" int svb_measure(svb_batch *b, const double *r, uint64_t *index) {
    if (!b || !r || !index) return SV_EINVAL;
    for (int i = 0; i < b->B; ++i)
        if (!(r[i] >= 0.0) || !std::isfinite(r[i])) return SV_EINVAL;
    if (int rc = ensure_red(b)) return rc;
    hipStream_t st = b->user_stream;
    double *dr = b->dred;                                              // B draws
    uint64_t *didx = reinterpret_cast<uint64_t *>(b->dred + b->B);    // B indices
    std::memcpy(b->hred, r, size_t(b->B) * sizeof(double));
    hipError_t e = hipMemcpyAsync(dr, b->hred, size_t(b->B) * sizeof(double), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
        const dim3 grid(unsigned(b->B)), blk(256);
        if (b->dtype == SV_C128)
            hipLaunchKernelGGL((k_measure_batch<c128>), grid, blk, 0, st, static_cast<const c128 *>(b->d), b->n, dr,
                               didx);
        else
            hipLaunchKernelGGL((k_measure_batch<c64>), grid, blk, 0, st, static_cast<const c64 *>(b->d), b->n, dr,
                               didx);
        e = hipGetLastError();
    }
    uint64_t *hidx = reinterpret_cast<uint64_t *>(b->hred + b->B);
    if (e == hipSuccess) e = hipMemcpyAsync(hidx, didx, size_t(b->B) * sizeof(uint64_t), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return svi_fail("svb_measure", e);
    std::memcpy(index, hidx, size_t(b->B) * sizeof(uint64_t));
    return SV_OK;
}

// ------------------------------------------------------------ no allocation
//
// svb_fidelity_noalloc: the per-register overlaps of svb_fidelity for
// callers that cannot allocate device memory.  Its partial sums (4 doubles
// per register) live in this file-scope device array instead of a
// hipMalloc'd buffer; each device holds its own copy until the process
// ends.  Host code reaches the array only through the address that
// hipGetSymbolAddress returns for the current device (the array's name is a
// host-side stand-in, not a device address).

static __device__ __align__(256) double scratch[SVB_NOALLOC_MAX_REGS * 4];

namespace {

// fid / overlap of each register from its four partial sums (re, im of
// <a|b>, |a|^2, |b|^2), as svb_fidelity forms them on the host.
__global__ __launch_bounds__(256) void k_fid_finish(const double *__restrict__ part, int nregs, double *__restrict__ fid,
                                                    double *__restrict__ overlap) {
    const int r = int(blockIdx.x) * 256 + int(threadIdx.x);
    if (r >= nregs) return;
    const double o0 = part[4 * r], o1 = part[4 * r + 1], o2 = part[4 * r + 2], o3 = part[4 * r + 3];
    if (overlap) {
        overlap[2 * r] = o0;
        overlap[2 * r + 1] = o1;
    }
    if (fid) fid[r] = (o2 > 0.0 && o3 > 0.0) ? (o0 * o0 + o1 * o1) / (o2 * o3) : 0.0;
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch[kMaxDevices] = {nullptr};

// Device address of the current device's scratch, looked up once per device.
int scratch_on_current_device(double **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return svi_fail("svb_fidelity_noalloc: current device", e);
    if (dev < 0 || dev >= kMaxDevices) return svi_fail_text("svb_fidelity_noalloc: device index out of range", SV_EDEVICE);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return svi_fail("svb_fidelity_noalloc: hipGetSymbolAddress", e);
        g_scratch[dev] = static_cast<double *>(p);
    }
    *out = g_scratch[dev];
    return SV_OK;
}

}  // namespace

extern "C" int svb_fidelity_noalloc(int n, int nregs, int dtype_a, const void *a, int dtype_b, const void *b,
                                    double *fid, double *overlap, void *hip_stream) {
    if (n < 1 || n > SV_MAX_QUBITS || !a || !b || (!fid && !overlap) || (dtype_a != SV_C64 && dtype_a != SV_C128) ||
        (dtype_b != SV_C64 && dtype_b != SV_C128))
        return SV_EINVAL;
    if (nregs < 1 || nregs > SVB_NOALLOC_MAX_REGS)
        return svi_fail_text("svb_fidelity_noalloc: nregs outside 1..SVB_NOALLOC_MAX_REGS", SV_EINVAL);
    double *part = nullptr;
    if (int rc = scratch_on_current_device(&part)) return rc;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    // every partial is written before it is read: nothing to clear
    const dim3 grid(static_cast<unsigned>(nregs)), blk(256);
    if (dtype_a == SV_C128 && dtype_b == SV_C128)
        hipLaunchKernelGGL((k_pair_overlap<c128, c128>), grid, blk, 0, st, static_cast<const c128 *>(a),
                           static_cast<const c128 *>(b), n, part);
    else if (dtype_a == SV_C128)
        hipLaunchKernelGGL((k_pair_overlap<c128, c64>), grid, blk, 0, st, static_cast<const c128 *>(a),
                           static_cast<const c64 *>(b), n, part);
    else if (dtype_b == SV_C128)
        hipLaunchKernelGGL((k_pair_overlap<c64, c128>), grid, blk, 0, st, static_cast<const c64 *>(a),
                           static_cast<const c128 *>(b), n, part);
    else
        hipLaunchKernelGGL((k_pair_overlap<c64, c64>), grid, blk, 0, st, static_cast<const c64 *>(a),
                           static_cast<const c64 *>(b), n, part);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_fid_finish, dim3(unsigned((nregs + 255) / 256)), dim3(256), 0, st, part, nregs, fid,
                           overlap);
        e = hipGetLastError();
    }
    return e == hipSuccess ? SV_OK : svi_fail("svb_fidelity_noalloc", e);
}
