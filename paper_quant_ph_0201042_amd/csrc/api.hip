// C ABI of the state-vector engine: argument validation, ownership, stream
// ordering and dispatch to the kernels.  Every argument check happens before
// any HIP call, so a rejected call enqueues nothing and needs no device.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "sv_internal.h"

int svi_status_from_hip(hipError_t e) {
    if (e == hipSuccess) return SV_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return SV_ENOMEM;
    return SV_EDEVICE;
}

namespace {
thread_local char g_last_error[256] = "";
}

int svi_fail(const char *what, hipError_t e) {
    if (e == hipSuccess) return SV_OK;
    std::snprintf(g_last_error, sizeof g_last_error, "%s: %s", what, hipGetErrorName(e));
    return svi_status_from_hip(e);
}

int svi_fail_text(const char *what, int status) {
    std::snprintf(g_last_error, sizeof g_last_error, "%s", what);
    return status;
}

extern "C" const char *sv_last_error(void) { return g_last_error; }

namespace {

bool valid_dtype(int d) { return d == SV_C64 || d == SV_C128; }
bool valid_n(int n) { return n >= 1 && n <= SV_MAX_QUBITS; }
uint64_t full_mask(int n) { return (uint64_t(1) << n) - 1; }

// Lazily allocated reduction scratch: wrapping a buffer needs no device call.
int ensure_scratch(sv_state *s) {
    if (!s->d_red) {
        hipError_t e = hipMalloc(reinterpret_cast<void **>(&s->d_red), SVI_RED_SLOTS * sizeof(double));
        if (e != hipSuccess) {
            s->d_red = nullptr;
            return svi_status_from_hip(e);
        }
    }
    if (!s->h_red) {
        hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&s->h_red), 4 * sizeof(double), hipHostMallocDefault);
        if (e != hipSuccess) {
            s->h_red = nullptr;
            return svi_status_from_hip(e);
        }
    }
    return SV_OK;
}

int finish_launch(hipError_t e) { return svi_status_from_hip(e); }

int sync_stream(hipStream_t st) {
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return SV_EDEVICE;
    e = hipGetLastError();
    return e == hipSuccess ? SV_OK : SV_EDEVICE;
}

// Checks a gate's qubits and controls against n (SWAP: two distinct-or-equal
// qubits, no controls).
bool gate_qubits_ok(int n, int q, uint64_t ctrl) {
    if (q < 0 || q >= n) return false;
    if (ctrl & ~full_mask(n)) return false;
    if (ctrl & (uint64_t(1) << (n - 1 - q))) return false;
    return true;
}

}  // namespace

extern "C" const char *sv_strerror(int status) {
    switch (status) {
    case SV_OK: return "ok";
    case SV_EINVAL: return "invalid argument";
    case SV_ENOMEM: return "device memory allocation failed";
    case SV_EDEVICE: return "HIP device or launch error";
    case SV_ENOTSUP: return "not supported";
    default: return "unknown status";
    }
}

extern "C" int sv_wrap(int n, int dtype, void *dev_ptr, void *hip_stream, sv_state **out) {
    if (!out) return SV_EINVAL;
    *out = nullptr;
    if (!valid_n(n) || !valid_dtype(dtype) || !dev_ptr) return SV_EINVAL;
    if (reinterpret_cast<uintptr_t>(dev_ptr) % dtype) return SV_EINVAL;
    sv_state *s = new (std::nothrow) sv_state;
    if (!s) return SV_ENOMEM;
    s->n = n;
    s->dtype = dtype;
    s->d = dev_ptr;
    s->owned = false;
    s->stream = static_cast<hipStream_t>(hip_stream);
    s->device = -1;
    s->d_red = nullptr;
    s->h_red = nullptr;
    s->fused = nullptr;
    s->prof = nullptr;
    s->adj = nullptr;
    s->work = nullptr;
    s->work_cap = 0;
    *out = s;
    return SV_OK;
}

extern "C" int sv_create(int n, int dtype, void *hip_stream, sv_state **out) {
    if (!out) return SV_EINVAL;
    *out = nullptr;
    if (!valid_n(n) || !valid_dtype(dtype)) return SV_EINVAL;
    void *d = nullptr;
    hipError_t e = hipMalloc(&d, (size_t(1) << n) * size_t(dtype));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return e == hipErrorOutOfMemory ? SV_ENOMEM : svi_status_from_hip(e);
    }
    int rc = sv_wrap(n, dtype, d, hip_stream, out);
    if (rc != SV_OK) {
        (void)hipFree(d);
        return rc;
    }
    (*out)->owned = true;
    rc = finish_launch(svi_launch_reset(*out, 0));
    if (rc != SV_OK) {
        sv_destroy(*out);
        *out = nullptr;
    }
    return rc;
}

extern "C" int sv_destroy(sv_state *s) {
    if (!s) return SV_OK;
    int rc = SV_OK;
    if (s->owned || s->d_red || s->h_red || s->work) {
        if (hipStreamSynchronize(s->stream) != hipSuccess) rc = SV_EDEVICE;
    }
    if (s->owned && s->d && hipFree(s->d) != hipSuccess) rc = SV_EDEVICE;
    if (s->work && hipFree(s->work) != hipSuccess) rc = SV_EDEVICE;
    if (s->d_red && hipFree(s->d_red) != hipSuccess) rc = SV_EDEVICE;
    if (s->h_red && hipHostFree(s->h_red) != hipSuccess) rc = SV_EDEVICE;
    svi_release_fused(s);
    svi_prof_release(s);
    svi_release_adjoint(s);
    delete s;
    return rc;
}

extern "C" int sv_set_stream(sv_state *s, void *hip_stream) {
    if (!s) return SV_EINVAL;
    s->stream = static_cast<hipStream_t>(hip_stream);
    return SV_OK;
}

extern "C" int sv_info(const sv_state *s, int *n, int *dtype, void **dev_ptr) {
    if (!s) return SV_EINVAL;
    if (n) *n = s->n;
    if (dtype) *dtype = s->dtype;
    if (dev_ptr) *dev_ptr = s->d;
    return SV_OK;
}

extern "C" int sv_reset(sv_state *s, uint64_t basis_index) {
    if (!s || basis_index > full_mask(s->n)) return SV_EINVAL;
    return finish_launch(svi_launch_reset(s, basis_index));
}

extern "C" int sv_load(sv_state *s, const void *src, int src_on_device) {
    if (!s || !src) return SV_EINVAL;
    const size_t bytes = (size_t(1) << s->n) * size_t(s->dtype);
    hipError_t e = hipMemcpyAsync(s->d, src, bytes, src_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                                  s->stream);
    if (e != hipSuccess) return SV_EDEVICE;
    if (!src_on_device) return sync_stream(s->stream);  // the host buffer may be reused at once
    return SV_OK;
}

extern "C" int sv_store(const sv_state *s, void *dst, int dst_on_device) {
    if (!s || !dst) return SV_EINVAL;
    const size_t bytes = (size_t(1) << s->n) * size_t(s->dtype);
    hipError_t e = hipMemcpyAsync(dst, s->d, bytes, dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                  s->stream);
    if (e != hipSuccess) return SV_EDEVICE;
    if (!dst_on_device) return sync_stream(s->stream);
    return SV_OK;
}

extern "C" int sv_apply_1q(sv_state *s, int q, const double U[8]) {
    if (!s || !U) return SV_EINVAL;
    if (!gate_qubits_ok(s->n, q, 0) || !svi_finite(U)) return SV_EINVAL;
    return finish_launch(svi_launch_gate(s, 0, q, U));
}

extern "C" int sv_apply_ctrl(sv_state *s, uint64_t ctrl_mask, int q, const double U[8]) {
    if (!s || !U) return SV_EINVAL;
    if (!gate_qubits_ok(s->n, q, ctrl_mask) || !svi_finite(U)) return SV_EINVAL;
    return finish_launch(svi_launch_gate(s, ctrl_mask, q, U));
}

extern "C" int sv_apply_swap(sv_state *s, int q1, int q2) {
    if (!s) return SV_EINVAL;
    if (q1 < 0 || q1 >= s->n || q2 < 0 || q2 >= s->n) return SV_EINVAL;
    return finish_launch(svi_launch_swap(s, q1, q2));
}

extern "C" int sv_prob(sv_state *s, uint64_t mask, uint64_t value, double *out) {
    if (!s || !out) return SV_EINVAL;
    if ((mask & ~full_mask(s->n)) || (value & ~mask)) return SV_EINVAL;
    int rc = ensure_scratch(s);
    if (rc != SV_OK) return rc;
    rc = finish_launch(svi_launch_prob(s, mask, value, s->d_red, s->d_red + 2 * SVI_RED_BLOCKS));
    if (rc != SV_OK) return rc;
    hipError_t e = hipMemcpyAsync(s->h_red, s->d_red + 2 * SVI_RED_BLOCKS, sizeof(double), hipMemcpyDeviceToHost,
                                  s->stream);
    if (e != hipSuccess) return SV_EDEVICE;
    rc = sync_stream(s->stream);
    if (rc != SV_OK) return rc;
    *out = s->h_red[0];
    return SV_OK;
}

// Measurement (sec. 2.2.3): the smallest i with sum_{j<i} |alpha_j|^2 <= r <
// sum_{j<=i} |alpha_j|^2, found by descending through chunk sums: at each
// level the range is split into at most SVI_RED_BLOCKS chunks whose FP64 sums
// are scanned on the host in index order; a range of at most 4096
// amplitudes is read and scanned directly.  Running sums are absolute
// (offsets are added, never subtracted).
extern "C" int sv_measure(sv_state *s, double r, uint64_t *index) {
    if (!s || !index || !(r >= 0.0) || !std::isfinite(r)) return SV_EINVAL;
    int rc = ensure_scratch(s);
    if (rc != SV_OK) return rc;
    const size_t w = size_t(s->dtype);
    uint64_t lo = 0, len = uint64_t(1) << s->n;
    double base = 0.0;     // sum of the weights before lo
    bool last_mode = false;  // r beyond the total: find the last nonzero weight
    std::vector<double> part(SVI_RED_BLOCKS);
    while (len > 4096) {
        const uint64_t chunk = std::max<uint64_t>(4096, len / SVI_RED_BLOCKS);
        const int nch = int(len / chunk);
        rc = finish_launch(svi_launch_chunk_sums(s, lo, chunk, nch, s->d_red));
        if (rc != SV_OK) return rc;
        hipError_t e = hipMemcpyAsync(part.data(), s->d_red, size_t(nch) * sizeof(double), hipMemcpyDeviceToHost,
                                      s->stream);
        if (e != hipSuccess) return svi_fail("sv_measure (copy)", e);
        rc = sync_stream(s->stream);
        if (rc != SV_OK) return rc;
        int pick = -1, lastnz = -1;
        double acc = base;
        for (int c = 0; c < nch; ++c) {
            if (part[size_t(c)] > 0.0) lastnz = c;
            if (!last_mode && pick < 0) {
                if (r < acc + part[size_t(c)]) {
                    pick = c;
                    base = acc;
                } else {
                    acc += part[size_t(c)];
                }
            }
        }
        if (pick < 0) {
            if (lastnz < 0) {  // no weight in this range (all-zero register)
                *index = lo;
                return SV_OK;
            }
            last_mode = true;
            pick = lastnz;
        }
        lo += uint64_t(pick) * chunk;
        len = chunk;
    }
    std::vector<char> buf(size_t(len) * w);
    hipError_t e = hipMemcpyAsync(buf.data(), static_cast<char *>(s->d) + lo * w, buf.size(), hipMemcpyDeviceToHost,
                                  s->stream);
    if (e != hipSuccess) return svi_fail("sv_measure (copy)", e);
    rc = sync_stream(s->stream);
    if (rc != SV_OK) return rc;
    double acc = base;
    uint64_t last = lo;
    for (uint64_t j = 0; j < len; ++j) {
        double re, im;
        if (s->dtype == SV_C128) {
            re = reinterpret_cast<const double *>(buf.data())[2 * j];
            im = reinterpret_cast<const double *>(buf.data())[2 * j + 1];
        } else {
            re = reinterpret_cast<const float *>(buf.data())[2 * j];
            im = reinterpret_cast<const float *>(buf.data())[2 * j + 1];
        }
        const double wt = re * re + im * im;
        if (wt > 0.0) last = lo + j;
        acc += wt;
        if (!last_mode && r < acc) {
            *index = lo + j;
            return SV_OK;
        }
    }
    *index = last;
    return SV_OK;
}

// Projective measurement outcome (sec. 2.2.3 with respect to the basis
// states of the qubits in mask): keeps the amplitudes with (j & mask) ==
// value, scaled by 1/sqrt(p) with p their total weight (FP64), and zeroes the
// rest.  p == 0 is rejected (SV_EINVAL) and leaves the register unchanged.
extern "C" int sv_collapse(sv_state *s, uint64_t mask, uint64_t value, double *prob) {
    if (!s) return SV_EINVAL;
    if ((mask & ~full_mask(s->n)) || (value & ~mask)) return SV_EINVAL;
    double p = 0.0;
    int rc = sv_prob(s, mask, value, &p);
    if (rc != SV_OK) return rc;
    if (!(p > 0.0)) return SV_EINVAL;
    rc = finish_launch(svi_launch_collapse(s, mask, value, 1.0 / std::sqrt(p)));
    if (rc != SV_OK) return rc;
    if (prob) *prob = p;
    return SV_OK;
}

extern "C" int sv_inner(sv_state *a, sv_state *b, double out[2]) {
    if (!a || !b || !out) return SV_EINVAL;
    if (a->n != b->n) return SV_EINVAL;
    int rc = ensure_scratch(b);
    if (rc != SV_OK) return rc;
    if (a->stream != b->stream) {
        // order a's pending work before the reduction on b's stream
        hipEvent_t ev;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return SV_EDEVICE;
        hipError_t e = hipEventRecord(ev, a->stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, ev, 0);
        (void)hipEventDestroy(ev);
        if (e != hipSuccess) return SV_EDEVICE;
    }
    rc = finish_launch(svi_launch_inner(a, b, b->stream, b->d_red, b->d_red + 2 * SVI_RED_BLOCKS));
    if (rc != SV_OK) return rc;
    hipError_t e = hipMemcpyAsync(b->h_red, b->d_red + 2 * SVI_RED_BLOCKS, 2 * sizeof(double),
                                  hipMemcpyDeviceToHost, b->stream);
    if (e != hipSuccess) return SV_EDEVICE;
    rc = sync_stream(b->stream);
    if (rc != SV_OK) return rc;
    out[0] = b->h_red[0];
    out[1] = b->h_red[1];
    return SV_OK;
}

extern "C" int sv_fidelity(sv_state *a, sv_state *b, double *fid) {
    if (!a || !b || !fid || a->n != b->n) return SV_EINVAL;
    double ab[2], aa, bb;
    int rc = sv_inner(a, b, ab);
    if (rc == SV_OK) rc = sv_prob(a, 0, 0, &aa);
    if (rc == SV_OK) rc = sv_prob(b, 0, 0, &bb);
    if (rc != SV_OK) return rc;
    if (!(aa > 0.0) || !(bb > 0.0)) return SV_EINVAL;
    *fid = (ab[0] * ab[0] + ab[1] * ab[1]) / (aa * bb);
    return SV_OK;
}

extern "C" int sv_overlap_loss(sv_state *phi, sv_state *psi, double *loss, double A[2]) {
    if (!phi || !psi || !loss) return SV_EINVAL;
    double ov[2];
    const int rc = sv_inner(phi, psi, ov);
    if (rc != SV_OK) return rc;
    *loss = 1.0 - (ov[0] * ov[0] + ov[1] * ov[1]);
    if (A) {
        A[0] = ov[0];
        A[1] = ov[1];
    }
    return SV_OK;
}

extern "C" int sv_sync(sv_state *s) {
    if (!s) return SV_EINVAL;
    return sync_stream(s->stream);
}

// ------------------------------------------------------------------ circuits

int svi_prepare(int n, const sv_gate *gates, int64_t ng, std::vector<PreparedGate> &out, int64_t *bad) {
    out.resize(size_t(ng));
    for (int64_t i = 0; i < ng; ++i) {
        const sv_gate &g = gates[i];
        PreparedGate &p = out[size_t(i)];
        p.kind = g.kind;
        p.q = g.target;
        p.q2 = g.target2;
        p.ctrl = g.ctrl;
        p.cls = GC_DENSE;
        bool ok;
        if (g.kind == SV_G_SWAP) {
            ok = g.ctrl == 0 && g.target >= 0 && g.target < n && g.target2 >= 0 && g.target2 < n;
        } else {
            ok = gate_qubits_ok(n, g.target, g.ctrl) && svi_gate_matrix(&g, p.U) == SV_OK && svi_finite(p.U);
            if (ok) p.cls = svi_classify(p.U);
        }
        if (!ok) {
            if (bad) *bad = i;
            return SV_EINVAL;
        }
    }
    return SV_OK;
}


extern "C" int sv_run(sv_state *s, const sv_gate *gates, int64_t ng, int flags, int64_t *bad_index) {
    if (bad_index) *bad_index = -1;
    if (!s || ng < 0 || (ng > 0 && !gates)) return SV_EINVAL;
    if (flags & ~(SV_RUN_FUSED | SV_RUN_PROFILE | SV_RUN_BLOCKS)) return SV_EINVAL;
    if ((flags & SV_RUN_FUSED) && (flags & SV_RUN_BLOCKS)) return SV_EINVAL;
    std::vector<PreparedGate> prep;
    int rc = svi_prepare(s->n, gates, ng, prep, bad_index);
    if (rc != SV_OK) return rc;
    const bool prof = (flags & SV_RUN_PROFILE) != 0;
    if (s->prof) s->prof->used = 0;
    if (flags & SV_RUN_FUSED) return svi_run_fused(s, prep.data(), ng, prof);
    if (flags & SV_RUN_BLOCKS) return svi_run_blocks(s, prep.data(), ng, prof);
    for (const PreparedGate &p : prep) {
        const int slot = svi_prof_begin(s, prof, p.kind == SV_G_SWAP ? STEP_SWAP : STEP_GATE);
        hipError_t e = p.kind == SV_G_SWAP ? svi_launch_swap(s, p.q, p.q2) : svi_launch_gate(s, p.ctrl, p.q, p.U);
        svi_prof_end(s, slot);
        if (e != hipSuccess) return svi_status_from_hip(e);
    }
    return SV_OK;
}

// The QFT of sec. 2.3.2 on qubits q0 .. q0 + m - 1 (qubit q0 the most
// significant bit of the sub-register index), run as fused passes: H on each
// qubit followed by R_k controlled by every later qubit, then the bit
// reversal by swaps (one permutation pass).  The inverse runs the adjoint
// gates in reverse order; R_k^dagger is R_k with its phase negated exactly
// (the deviation -2 * 2 pi / 2^k added to 2 pi / 2^k).
extern "C" int sv_qft(sv_state *s, int q0, int m, int flags) {
    if (!s || q0 < 0 || m < 1 || q0 + m > s->n) return SV_EINVAL;
    if (flags & ~(SV_QFT_INVERSE | SV_QFT_BITREV)) return SV_EINVAL;
    const bool inverse = flags & SV_QFT_INVERSE, swaps = !(flags & SV_QFT_BITREV);
    if (svi_config().qft_fft && svi_qft_fft_ok(s)) {
        // FFT block passes leave the range bit-reversed: QFT = R G+, inverse =
        // R G-, inverse reading a bit-reversed input = R G- R (R the reversal)
        const int lo = s->n - q0 - m;
        int f[64];
        for (int b = 0; b < s->n; ++b) f[b] = (b >= lo && b < lo + m) ? 2 * lo + m - 1 - b : b;
        auto reverse = [&]() { return m < 2 ? SV_OK : finish_launch(svi_launch_bitperm(s, f)); };
        int rc = SV_OK;
        if (inverse && !swaps) rc = reverse();
        if (rc == SV_OK) rc = svi_qft_fft(s, lo, m, inverse ? -1 : +1);
        if (rc == SV_OK && (swaps || inverse)) rc = reverse();
        return rc;
    }
    const int n = s->n;
    auto bit = [&](int q) { return uint64_t(1) << (n - 1 - q); };
    std::vector<sv_gate> g;
    auto add = [&](int kind, int q, uint64_t ctrl, int q2, int iarg, double phase_dev) {
        sv_gate x;
        std::memset(&x, 0, sizeof x);
        x.kind = kind;
        x.target = q;
        x.target2 = q2;
        x.iarg = iarg;
        x.ctrl = ctrl;
        x.p[1] = phase_dev;
        g.push_back(x);
    };
    const double two_pi = 6.283185307179586476925286766559;
    if (!inverse) {
        for (int i = 0; i < m; ++i) {
            add(SV_G_H, q0 + i, 0, -1, 0, 0.0);
            for (int c = i + 1; c < m; ++c) add(SV_G_RK, q0 + i, bit(q0 + c), -1, c - i + 1, 0.0);
        }
        if (swaps)
            for (int i = 0; i < m / 2; ++i) add(SV_G_SWAP, q0 + i, 0, q0 + m - 1 - i, 0, 0.0);
    } else {
        if (swaps)
            for (int i = 0; i < m / 2; ++i) add(SV_G_SWAP, q0 + i, 0, q0 + m - 1 - i, 0, 0.0);
        for (int i = m - 1; i >= 0; --i) {
            for (int c = m - 1; c > i; --c)
                add(SV_G_RK, q0 + i, bit(q0 + c), -1, c - i + 1, -2.0 * (two_pi / std::ldexp(1.0, c - i + 1)));
            add(SV_G_H, q0 + i, 0, -1, 0, 0.0);
        }
    }
    return sv_run(s, g.data(), int64_t(g.size()), SV_RUN_FUSED, nullptr);
}

// ------------------------------------------------------------------ tuning

// Engine parameters, process-wide (field order of SviConfig).
SviConfig &svi_config() {
    static SviConfig c = {12, 12, 4, 512, 5, 1, 1, 1, 6, 16384, 1, 4, 384, 1, 256, 0, 1, 5, 0, 1, 1, 4, 1, 4};
    return c;
}

namespace {
struct ConfigKey {
    const char *name;
    int SviConfig::*field;
    int lo, hi;
};
const ConfigKey kKeys[] = {
    {"fused_tile_bits_c128", &SviConfig::fused_tile_bits_c128, 1, 12},
    {"fused_tile_bits_c64", &SviConfig::fused_tile_bits_c64, 1, 13},
    {"fused_low_bits", &SviConfig::fused_low_bits, 1, 12},
    {"fused_max_ops", &SviConfig::fused_max_ops, 1, 4096},
    {"block_qubits", &SviConfig::block_qubits, 1, 6},
    {"fused_jit", &SviConfig::fused_jit, 0, 1},
    {"fused_pairs", &SviConfig::fused_pairs, 0, 1},
    {"swap_runs", &SviConfig::swap_runs, 0, 1},
    {"perm_low_bits", &SviConfig::perm_low_bits, 1, 6},
    {"perm_workgroups", &SviConfig::perm_workgroups, 1, 1 << 20},
    {"fused_plan_search", &SviConfig::fused_plan_search, 0, 1},
    {"fused_reg_bits", &SviConfig::fused_reg_bits, 2, 4},
    {"fused_jit_max_ops", &SviConfig::fused_jit_max_ops, 1, 4096},
    {"qft_fft", &SviConfig::qft_fft, 0, 1},
    {"mfma_workgroups", &SviConfig::mfma_workgroups, 1, 1 << 20},
    {"fused_mfma", &SviConfig::fused_mfma, 0, 1},
    {"fused_rotations", &SviConfig::fused_rotations, 0, 1},
    {"perm_low_bits_c64", &SviConfig::perm_low_bits_c64, 1, 6},
    {"gate_pairs_min_bit", &SviConfig::gate_pairs_min_bit, 0, 6},
    {"gate_cached_low", &SviConfig::gate_cached_low, 0, 1},
    {"batch_mfma", &SviConfig::batch_mfma, 0, 1},
    {"batch_waves", &SviConfig::batch_waves, 0, 8},
    {"batch_const_bits", &SviConfig::batch_const_bits, 0, 1},
    {"gate_spread_bits", &SviConfig::gate_spread_bits, 0, 8},
};
const ConfigKey *find_key(const char *key) {
    if (!key) return nullptr;
    for (const ConfigKey &k : kKeys)
        if (std::strcmp(k.name, key) == 0) return &k;
    return nullptr;
}
}  // namespace

extern "C" int sv_config_set(const char *key, int value) {
    const ConfigKey *k = find_key(key);
    if (!k || value < k->lo || value > k->hi) return SV_EINVAL;
    svi_config().*(k->field) = value;
    return SV_OK;
}

extern "C" int sv_config_get(const char *key, int *value) {
    const ConfigKey *k = find_key(key);
    if (!k || !value) return SV_EINVAL;
    *value = svi_config().*(k->field);
    return SV_OK;
}

// ------------------------------------------------------------------ profiling

int svi_prof_begin(sv_state *s, bool on, int kind) {
    if (!on) return -1;
    if (!s->prof) s->prof = new (std::nothrow) RunProfile();
    if (!s->prof) return -1;
    RunProfile &p = *s->prof;
    const size_t slot = p.used;
    if (p.ev.size() < 2 * (slot + 1)) {
        hipEvent_t e0, e1;
        if (hipEventCreate(&e0) != hipSuccess) return -1;
        if (hipEventCreate(&e1) != hipSuccess) {
            (void)hipEventDestroy(e0);
            return -1;
        }
        p.ev.push_back(e0);
        p.ev.push_back(e1);
    }
    if (p.kind.size() < slot + 1) p.kind.resize(slot + 1);
    p.kind[slot] = kind;
    if (hipEventRecord(p.ev[2 * slot], s->stream) != hipSuccess) return -1;
    p.used = slot + 1;
    return int(slot);
}

void svi_prof_end(sv_state *s, int slot) {
    if (slot < 0 || !s->prof) return;
    (void)hipEventRecord(s->prof->ev[2 * size_t(slot) + 1], s->stream);
}

void svi_prof_release(sv_state *s) {
    if (!s->prof) return;
    for (hipEvent_t e : s->prof->ev) (void)hipEventDestroy(e);
    delete s->prof;
    s->prof = nullptr;
}

extern "C" int sv_run_profile(sv_state *s, double *ms, int32_t *kind, int64_t cap, int64_t *count) {
    if (!s || !count || cap < 0) return SV_EINVAL;
    *count = 0;
    if (!s->prof) return SV_OK;
    RunProfile &p = *s->prof;
    const int64_t nsteps = int64_t(p.used);
    *count = nsteps;
    for (int64_t i = 0; i < nsteps && i < cap; ++i) {
        if (hipEventSynchronize(p.ev[2 * size_t(i) + 1]) != hipSuccess) return SV_EDEVICE;
        float t = 0.f;
        if (hipEventElapsedTime(&t, p.ev[2 * size_t(i)], p.ev[2 * size_t(i) + 1]) != hipSuccess) return SV_EDEVICE;
        if (ms) ms[i] = double(t);
        if (kind) kind[i] = p.kind[size_t(i)];
    }
    return SV_OK;
}
