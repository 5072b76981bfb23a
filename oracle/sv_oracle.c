/*
 * Plain, single-threaded FP64 reference simulator ("the oracle").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this file's library.  It shares no
 * code with the HIP library: no headers, no helpers, no tables.
 *
 * Built with: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared (no fast-math,
 * no SIMD intrinsics, no threads), so every sum is evaluated in source order.
 *
 * Conventions (Niwa-Matsumoto-Imai, sec. 2.1 Registers and 2.2.1):
 *   - a register of n qubits is 2^n complex doubles, alpha_j, j = basis index;
 *   - qubit 0 is the most significant bit, so qubit q is index bit b = n-1-q;
 *   - a 2x2 matrix U is 8 doubles: u11re,u11im,u12re,u12im,u21re,u21im,u22re,u22im.
 *
 * Every function below cites the passage of the paper it follows.  Parity
 * pins live in tests/test_oracle_*.py.  One function has no external pin and
 * says so: orc_noisy_grover_traj and orc_noisy_traj_state (their draw
 * schedule is this project's reading; their gate semantics are pinned through
 * orc_gate_matrix and orc_run).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double re, im;
} cplx;

static cplx c_make(double re, double im) {
    cplx z;
    z.re = re;
    z.im = im;
    return z;
}
static cplx c_add(cplx a, cplx b) { return c_make(a.re + b.re, a.im + b.im); }
static cplx c_mul(cplx a, cplx b) {
    return c_make(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
static cplx c_conj(cplx a) { return c_make(a.re, -a.im); }

/* Gate record, one per gate of a serialized gate list (88 bytes). */
typedef struct {
    int32_t kind;
    int32_t target;
    int32_t target2;
    int32_t iarg;
    uint64_t ctrl;
    double p[8];
} orc_gate;

enum { K_U = 0, K_H, K_X, K_Y, K_Z, K_RK, K_ROT, K_SU2, K_SWAP };

static const double PI = 3.14159265358979323846;

/* ------------------------------------------------------------------ a9 ---
 * Gate matrices.  sec. 3.2 (Operational Error): every one-qubit gate is a
 * rotation U_R(theta) = [[cos, -sin], [sin, cos]] times a phase shift
 * U_P1(phi) = diag(1, e^{i phi}); H = U_R(pi/4) U_P1(pi) and
 * NOT = U_R(pi/2) U_P1(pi); errors are added to theta and phi.
 * Exact gates (both deviations zero) use their textbook entries, so that an
 * unperturbed NOT is a pure permutation.
 * R_k = diag(1, e^{2 pi i / 2^k}) (sec. 2.3.2 writes R_d with pi/2^d, d=k-1).
 */
static void set_u(double *U, cplx a, cplx b, cplx c, cplx d) {
    U[0] = a.re; U[1] = a.im; U[2] = b.re; U[3] = b.im;
    U[4] = c.re; U[5] = c.im; U[6] = d.re; U[7] = d.im;
}

static void rot_phase(double theta, double phi, double *U) {
    /* U_R(theta) U_P1(phi) = [[cos, -sin e^{i phi}], [sin, cos e^{i phi}]] */
    double c = cos(theta), s = sin(theta);
    cplx e = c_make(cos(phi), sin(phi));
    set_u(U, c_make(c, 0.0), c_make(-s * e.re, -s * e.im),
          c_make(s, 0.0), c_make(c * e.re, c * e.im));
}

static void phase_only(double phi, double *U) {
    set_u(U, c_make(1.0, 0.0), c_make(0.0, 0.0), c_make(0.0, 0.0),
          c_make(cos(phi), sin(phi)));
}

int orc_gate_matrix(int kind, int iarg, const double *p, double *U) {
    switch (kind) {
    case K_U:
        memcpy(U, p, 8 * sizeof(double));
        return 0;
    case K_H:
        if (p[0] == 0.0 && p[1] == 0.0) {
            double r = sqrt(0.5);
            set_u(U, c_make(r, 0), c_make(r, 0), c_make(r, 0), c_make(-r, 0));
        } else {
            rot_phase(PI / 4 + p[0], PI + p[1], U);
        }
        return 0;
    case K_X:
        if (p[0] == 0.0 && p[1] == 0.0)
            set_u(U, c_make(0, 0), c_make(1, 0), c_make(1, 0), c_make(0, 0));
        else
            rot_phase(PI / 2 + p[0], PI + p[1], U);
        return 0;
    case K_Y:
        set_u(U, c_make(0, 0), c_make(0, -1), c_make(0, 1), c_make(0, 0));
        return 0;
    case K_Z:
        if (p[1] == 0.0)
            set_u(U, c_make(1, 0), c_make(0, 0), c_make(0, 0), c_make(-1, 0));
        else
            phase_only(PI + p[1], U);
        return 0;
    case K_RK:
        if (iarg < 0 || iarg > 62) return -1;
        phase_only(2.0 * PI / ldexp(1.0, iarg) + p[1], U);
        return 0;
    case K_ROT:
        rot_phase(p[0], p[1], U);
        return 0;
    case K_SU2: {
        /* Haar SU(2) from a Gaussian quaternion (q0,q1,q2,q3) normalised to 1:
           [[q0 + i q1, q2 + i q3], [-q2 + i q3, q0 - i q1]] */
        double nrm = sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2] + p[3] * p[3]);
        if (!(nrm > 0.0)) return -1;
        double a = p[0] / nrm, b = p[1] / nrm, c = p[2] / nrm, d = p[3] / nrm;
        set_u(U, c_make(a, b), c_make(c, d), c_make(-c, d), c_make(a, -b));
        return 0;
    }
    default:
        return -1;
    }
}

/* Derivative of a gate matrix with respect to one of its angle deviations
 * (which = 0: theta deviation p[0]; which = 1: phi deviation p[1]).  Used by
 * the adjoint reference.  d/dtheta U_R = [[-sin, -cos], [cos, -sin]];
 * d/dphi U_P1 = diag(0, i e^{i phi}).  Returns -1 for a kind with no such
 * parameter. */
int orc_gate_dmatrix(int kind, int iarg, const double *p, int which, double *D) {
    double theta, phi;
    int has_rot;
    switch (kind) {
    case K_H: theta = PI / 4 + p[0]; phi = PI + p[1]; has_rot = 1; break;
    case K_X: theta = PI / 2 + p[0]; phi = PI + p[1]; has_rot = 1; break;
    case K_ROT: theta = p[0]; phi = p[1]; has_rot = 1; break;
    case K_Z: theta = 0; phi = PI + p[1]; has_rot = 0; break;
    case K_RK:
        if (iarg < 0 || iarg > 62) return -1;
        theta = 0; phi = 2.0 * PI / ldexp(1.0, iarg) + p[1]; has_rot = 0; break;
    default: return -1;
    }
    cplx e = c_make(cos(phi), sin(phi));
    cplx ie = c_make(-sin(phi), cos(phi)); /* i e^{i phi} */
    if (which == 0) {
        if (!has_rot) return -1;
        double c = cos(theta), s = sin(theta);
        /* dU_R(theta) U_P1(phi) = [[-s, -c e], [c, -s e]] */
        set_u(D, c_make(-s, 0), c_make(-c * e.re, -c * e.im), c_make(c, 0),
              c_make(-s * e.re, -s * e.im));
        return 0;
    }
    if (which == 1) {
        if (has_rot) {
            double c = cos(theta), s = sin(theta);
            /* U_R(theta) dU_P1(phi) = [[0, -s ie], [0, c ie]] */
            set_u(D, c_make(0, 0), c_make(-s * ie.re, -s * ie.im), c_make(0, 0),
                  c_make(c * ie.re, c * ie.im));
        } else {
            set_u(D, c_make(0, 0), c_make(0, 0), c_make(0, 0), ie);
        }
        return 0;
    }
    return -1;
}

/* ------------------------------------------------------------ a2, a3 ---
 * sec. 2.2.1: a one-qubit gate on qubit q changes each pair of rows
 * (j, j + 2^{n-q-1}) with j's bit of qubit q equal to 0:
 *   x' = u11 x + u12 y,  y' = u21 x + u22 y.
 * The first result goes to a temporary so the second still reads the old x
 * (the in-place hazard the paper describes in its Parallelization paragraph).
 * sec. 2.2.2: with controls, rows whose control bits are not all 1 are left
 * alone (CTX[j] = I[j]).  A mask of several controls is the many-controlled
 * extension the same passage mentions.
 * An exact NOT matrix is applied as a swap of the two amplitudes, so that
 * permutation gates move values without arithmetic.
 */
static int is_exact_not(const double *U) {
    return U[0] == 0.0 && U[1] == 0.0 && U[2] == 1.0 && U[3] == 0.0 &&
           U[4] == 1.0 && U[5] == 0.0 && U[6] == 0.0 && U[7] == 0.0;
}

void orc_apply_ctrl(cplx *a, int n, uint64_t ctrl, int q, const double *U) {
    uint64_t N = (uint64_t)1 << n;
    uint64_t s = (uint64_t)1 << (n - 1 - q);
    cplx u11 = c_make(U[0], U[1]), u12 = c_make(U[2], U[3]);
    cplx u21 = c_make(U[4], U[5]), u22 = c_make(U[6], U[7]);
    int perm = is_exact_not(U);
    for (uint64_t base = 0; base < N; base += 2 * s) {
        for (uint64_t j = base; j < base + s; ++j) {
            if ((j & ctrl) != ctrl) continue;
            cplx x = a[j], y = a[j + s];
            if (perm) {
                a[j] = y;
                a[j + s] = x;
                continue;
            }
            cplx t = c_add(c_mul(u11, x), c_mul(u12, y));
            a[j + s] = c_add(c_mul(u21, x), c_mul(u22, y));
            a[j] = t;
        }
    }
}

void orc_apply_1q(cplx *a, int n, int q, const double *U) {
    orc_apply_ctrl(a, n, 0, q, U);
}

/* Exchange of two qubits (a permutation of basis states): amplitudes whose
 * bits for q1 and q2 differ trade places.  Used by the QFT's final swaps. */
void orc_swap(cplx *a, int n, int q1, int q2) {
    if (q1 == q2) return;
    uint64_t N = (uint64_t)1 << n;
    uint64_t m1 = (uint64_t)1 << (n - 1 - q1), m2 = (uint64_t)1 << (n - 1 - q2);
    for (uint64_t j = 0; j < N; ++j) {
        if ((j & m1) && !(j & m2)) {
            uint64_t k = (j & ~m1) | m2;
            cplx t = a[j];
            a[j] = a[k];
            a[k] = t;
        }
    }
}

/* Controlled derivative application used by the adjoint reference:
 * out = dCTX a, where dCTX has rows dX[j] when all control bits of j are 1
 * and zero rows otherwise (the identity rows of CTX do not depend on the
 * angle). */
void orc_apply_ctrl_derivative(cplx *a, int n, uint64_t ctrl, int q, const double *D) {
    uint64_t N = (uint64_t)1 << n;
    uint64_t s = (uint64_t)1 << (n - 1 - q);
    cplx d11 = c_make(D[0], D[1]), d12 = c_make(D[2], D[3]);
    cplx d21 = c_make(D[4], D[5]), d22 = c_make(D[6], D[7]);
    for (uint64_t base = 0; base < N; base += 2 * s) {
        for (uint64_t j = base; j < base + s; ++j) {
            if ((j & ctrl) != ctrl) {
                a[j] = c_make(0, 0);
                a[j + s] = c_make(0, 0);
                continue;
            }
            cplx x = a[j], y = a[j + s];
            cplx t = c_add(c_mul(d11, x), c_mul(d12, y));
            a[j + s] = c_add(c_mul(d21, x), c_mul(d22, y));
            a[j] = t;
        }
    }
}

/* ---------------------------------------------------------------- a5 ---
 * A dense k-qubit gate: the definition X = I (x) ... (x) M (x) ... (x) I of
 * sec. 2.2.1 generalised to a 2^k x 2^k block M on qubits qs[0..k-1].  The
 * local row index r has qs[0] as its most significant bit.  For every basis
 * index j whose k target bits are 0 the 2^k amplitudes j + offset(r) are
 * gathered, multiplied by M (row-major, complex interleaved) and scattered.
 */
int orc_apply_kq(cplx *a, int n, int k, const int *qs, const double *M) {
    if (k < 1 || k > 10) return -1;
    uint64_t N = (uint64_t)1 << n;
    uint64_t tmask = 0;
    int K = 1 << k;
    uint64_t *off = (uint64_t *)malloc(sizeof(uint64_t) * K);
    cplx *v = (cplx *)malloc(sizeof(cplx) * K);
    cplx *w = (cplx *)malloc(sizeof(cplx) * K);
    for (int i = 0; i < k; ++i) tmask |= (uint64_t)1 << (n - 1 - qs[i]);
    for (int r = 0; r < K; ++r) {
        uint64_t o = 0;
        for (int i = 0; i < k; ++i)
            if ((r >> (k - 1 - i)) & 1) o |= (uint64_t)1 << (n - 1 - qs[i]);
        off[r] = o;
    }
    for (uint64_t j = 0; j < N; ++j) {
        if (j & tmask) continue;
        for (int r = 0; r < K; ++r) v[r] = a[j + off[r]];
        for (int r = 0; r < K; ++r) {
            cplx acc = c_make(0, 0);
            for (int c = 0; c < K; ++c) {
                cplx m = c_make(M[2 * (r * K + c)], M[2 * (r * K + c) + 1]);
                acc = c_add(acc, c_mul(m, v[c]));
            }
            w[r] = acc;
        }
        for (int r = 0; r < K; ++r) a[j + off[r]] = w[r];
    }
    free(off);
    free(v);
    free(w);
    return 0;
}

/* ---------------------------------------------------------------- a6 ---
 * sec. 2.2.3 (Measurement Gates): the probability weights are |alpha_j|^2.
 * orc_prob sums them, in index order, over the basis states whose masked
 * bits equal `value`; orc_inner is <a|b> = sum_j conj(a_j) b_j in index order.
 */
double orc_prob(const cplx *a, int n, uint64_t mask, uint64_t value) {
    uint64_t N = (uint64_t)1 << n;
    double s = 0.0;
    for (uint64_t j = 0; j < N; ++j)
        if ((j & mask) == value) s += a[j].re * a[j].re + a[j].im * a[j].im;
    return s;
}

void orc_inner(const cplx *a, const cplx *b, int n, double *out) {
    uint64_t N = (uint64_t)1 << n;
    cplx s = c_make(0, 0);
    for (uint64_t j = 0; j < N; ++j) s = c_add(s, c_mul(c_conj(a[j]), b[j]));
    out[0] = s.re;
    out[1] = s.im;
}

/* sec. 2.2.3: draw r in [0,1) and return the i with
 * sum_{j<i} |alpha_j|^2 <= r < sum_{j<=i} |alpha_j|^2, scanning in index
 * order.  If rounding leaves r at or above the final sum, the last index with
 * nonzero weight is returned. */
uint64_t orc_measure(const cplx *a, int n, double r) {
    uint64_t N = (uint64_t)1 << n;
    double s = 0.0;
    uint64_t last = 0;
    for (uint64_t j = 0; j < N; ++j) {
        double w = a[j].re * a[j].re + a[j].im * a[j].im;
        if (w > 0.0) last = j;
        s += w;
        if (r < s) return j;
    }
    return last;
}

/* sec. 2.2.3 with respect to the basis states of the qubits in mask (a
 * basis-index mask): the outcome value has probability p = sum of
 * |alpha_j|^2 over j with (j & mask) == value (sequential FP64 sum); the
 * post-measurement register keeps those amplitudes divided by sqrt(p) and
 * sets the others to 0.  Returns p; p == 0 leaves the register unchanged. */
double orc_collapse(cplx *a, int n, uint64_t mask, uint64_t value) {
    uint64_t N = (uint64_t)1 << n;
    double p = 0.0;
    for (uint64_t j = 0; j < N; ++j)
        if ((j & mask) == value) p += a[j].re * a[j].re + a[j].im * a[j].im;
    if (!(p > 0.0)) return p;
    double scale = 1.0 / sqrt(p);
    for (uint64_t j = 0; j < N; ++j) {
        if ((j & mask) == value) {
            a[j].re *= scale;
            a[j].im *= scale;
        } else {
            a[j].re = 0.0;
            a[j].im = 0.0;
        }
    }
    return p;
}

/* ----------------------------------------------------------- circuits ---
 * Applies a serialized gate list in order (sec. 2.2: a circuit is a sequence
 * of evolution steps).  Returns the index of the first bad gate + 1, or 0.
 */
static int check_gate(const orc_gate *g, int n) {
    if (g->target < 0 || g->target >= n) return -1;
    uint64_t full = (n == 64) ? ~(uint64_t)0 : (((uint64_t)1 << n) - 1);
    if (g->ctrl & ~full) return -1;
    if (g->kind == K_SWAP) {
        if (g->target2 < 0 || g->target2 >= n || g->ctrl) return -1;
        return 0;
    }
    if (g->ctrl & ((uint64_t)1 << (n - 1 - g->target))) return -1;
    return 0;
}

int orc_apply_gate(cplx *a, int n, const orc_gate *g) {
    if (check_gate(g, n)) return -1;
    if (g->kind == K_SWAP) {
        orc_swap(a, n, g->target, g->target2);
        return 0;
    }
    double U[8];
    if (orc_gate_matrix(g->kind, g->iarg, g->p, U)) return -1;
    orc_apply_ctrl(a, n, g->ctrl, g->target, U);
    return 0;
}

int orc_run(cplx *a, int n, const orc_gate *gates, int64_t ng) {
    for (int64_t i = 0; i < ng; ++i)
        if (orc_apply_gate(a, n, &gates[i])) return (int)(i + 1);
    return 0;
}

/* Inverse of one gate: U^dagger on the same qubits (SWAP is its own inverse). */
int orc_apply_gate_inverse(cplx *a, int n, const orc_gate *g) {
    if (check_gate(g, n)) return -1;
    if (g->kind == K_SWAP) {
        orc_swap(a, n, g->target, g->target2);
        return 0;
    }
    double U[8], V[8];
    if (orc_gate_matrix(g->kind, g->iarg, g->p, U)) return -1;
    /* V = U^dagger: v11 = conj(u11), v12 = conj(u21), v21 = conj(u12), v22 = conj(u22) */
    V[0] = U[0]; V[1] = -U[1];
    V[2] = U[4]; V[3] = -U[5];
    V[4] = U[2]; V[5] = -U[3];
    V[6] = U[6]; V[7] = -U[7];
    orc_apply_ctrl(a, n, g->ctrl, g->target, V);
    return 0;
}

/* ------------------------------------------------------------ Philox ---
 * Philox4x32-10 counter-based generator, from its published definition
 * (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
 * SC'11): ten rounds of
 *   (hi0, lo0) = M0 * c0, (hi1, lo1) = M1 * c2,
 *   c = (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0),
 * with the key bumped by the Weyl constants between rounds.
 */
void orc_philox4x32_10(const uint32_t *ctr, const uint32_t *key, uint32_t *out) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* ------------------------------------------------------------ a7 -------
 * One noisy Grover trajectory (sec. 3 Error Model; sec. 5.3.1 Effect of
 * Errors): the ancilla-free Grover circuit for `marked`, in which
 *   - every gate's angles are perturbed (sec. 3.2): H, NOT and U_R U_P1
 *     rotations as U_R(theta0 + x) U_P1(phi0 + y); phase-shift gates (Z,
 *     R_k, the phase of a C^{n-1}Z) as phi0 + y; x, y ~ N(0, sigma^2);
 *     gates given as explicit matrices (U, SU2, Y) carry no angle;
 *   - after every gate, each qubit the gate touches (target and controls)
 *     independently suffers sigma_x, sigma_y or sigma_z with probability p/3
 *     each (sec. 3.1 depolarizing channel).
 * Draws (this project's reading; the paper does not fix a generator):
 *   key = (seed lo, seed hi); gate g of the trajectory, slot s:
 *   ctr = (traj, g, s, 0).
 *   slot 0: u_i = (r_i + 0.5) 2^-32; rad = sqrt(-2 ln u0);
 *           x = sigma rad cos(2 pi u1), y = sigma rad sin(2 pi u1).
 *   touched qubit number i (ascending qubit order) uses slot 1 + i/2, words
 *   2(i%2) (event: r < floor(p 2^32)) and 2(i%2)+1 (type: (3 r) >> 32,
 *   0 = sigma_x, 1 = sigma_y, 2 = sigma_z).
 * parity unpinned for the draw schedule itself (a reading, not a published
 * value); its noise-free limit, its gate semantics and its statistics are
 * pinned in the tests.
 * Returns |alpha_marked|^2 at the end, and writes the final state to `out`
 * when out != NULL.
 */
static void draw_slot(uint64_t seed, uint64_t traj, uint64_t g, uint32_t slot, uint32_t *r) {
    uint32_t ctr[4] = {(uint32_t)traj, (uint32_t)g, slot, 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, r);
}

static void noisy_gate(cplx *a, int n, const orc_gate *g, uint64_t gi, double sigma,
                       uint32_t pthresh, uint64_t seed, uint64_t traj, uint32_t depol_kinds) {
    orc_gate pg = *g;
    if (sigma != 0.0) {
        uint32_t r[4];
        draw_slot(seed, traj, gi, 0, r);
        double u0 = ((double)r[0] + 0.5) * ldexp(1.0, -32);
        double u1 = ((double)r[1] + 0.5) * ldexp(1.0, -32);
        double rad = sqrt(-2.0 * log(u0));
        double x = sigma * rad * cos(2.0 * PI * u1);
        double y = sigma * rad * sin(2.0 * PI * u1);
        if (pg.kind == K_H || pg.kind == K_X || pg.kind == K_ROT) {
            pg.p[0] += x; /* rotation angle */
            pg.p[1] += y; /* phase angle */
        } else if (pg.kind == K_Z || pg.kind == K_RK) {
            pg.p[1] += y; /* phase-shift gates: U_P1(phi) */
        }
    }
    orc_apply_gate(a, n, &pg);
    if (pthresh == 0 || !((depol_kinds >> g->kind) & 1u)) return;
    /* touched qubits in ascending qubit order */
    int i = 0;
    for (int q = 0; q < n; ++q) {
        uint64_t bit = (uint64_t)1 << (n - 1 - q);
        if (q != g->target && !(g->ctrl & bit)) continue;
        uint32_t r[4];
        draw_slot(seed, traj, gi, 1u + (uint32_t)(i / 2), r);
        uint32_t ev = r[2 * (i % 2)], ty = r[2 * (i % 2) + 1];
        ++i;
        if (ev >= pthresh) continue;
        int t = (int)(((uint64_t)ty * 3u) >> 32);
        orc_gate pauli;
        memset(&pauli, 0, sizeof pauli);
        pauli.kind = t == 0 ? K_X : (t == 1 ? K_Y : K_Z);
        pauli.target = q;
        pauli.target2 = -1;
        orc_apply_gate(a, n, &pauli);
    }
}

uint32_t orc_pauli_threshold(double p) {
    if (!(p > 0.0)) return 0;
    if (p >= 1.0) return 0xFFFFFFFFu;
    return (uint32_t)floor(p * 4294967296.0);
}

/* The same trajectory applied to a register given by the caller (in place),
 * for experiments that do not start from |0...0> (the QFT of sec. 5.1.1 acts
 * on the register left by the modular exponentiation).  Depolarizing draws
 * follow only the gates whose kind k has bit k set in depol_kinds: sec. 5.1.1
 * depolarizes the register each time an R_d is applied, which a gate list
 * expresses with explicit identity gates on every qubit after each R_d and
 * depol_kinds selecting those alone. */
void orc_noisy_traj_state(cplx *a, int n, int iters, double sigma, double p, uint64_t seed,
                          uint64_t traj, const orc_gate *init, int64_t n_init,
                          const orc_gate *iter, int64_t n_iter, uint32_t depol_kinds) {
    uint32_t pt = orc_pauli_threshold(p);
    uint64_t gi = 0;
    for (int64_t i = 0; i < n_init; ++i)
        noisy_gate(a, n, &init[i], gi++, sigma, pt, seed, traj, depol_kinds);
    for (int it = 0; it < iters; ++it)
        for (int64_t i = 0; i < n_iter; ++i)
            noisy_gate(a, n, &iter[i], gi++, sigma, pt, seed, traj, depol_kinds);
}

double orc_noisy_grover_traj(int n, uint64_t marked, int iters, double sigma, double p,
                             uint64_t seed, uint64_t traj, const orc_gate *init, int64_t n_init,
                             const orc_gate *iter, int64_t n_iter, cplx *out) {
    uint64_t N = (uint64_t)1 << n;
    cplx *a = out ? out : (cplx *)malloc(sizeof(cplx) * N);
    memset(a, 0, sizeof(cplx) * N);
    a[0] = c_make(1.0, 0.0);
    orc_noisy_traj_state(a, n, iters, sigma, p, seed, traj, init, n_init, iter, n_iter, 0xFFFFFFFFu);
    double pr = a[marked].re * a[marked].re + a[marked].im * a[marked].im;
    if (!out) free(a);
    return pr;
}

/* ------------------------------------------------------------ a8 -------
 * Adjoint gradient of loss = 1 - |<phi|psi(eps)>|^2, psi(eps) = U_L..U_1 psi0,
 * with respect to one angle deviation per gate (dparam[g] = 0: theta,
 * 1: phi, -1: none).  Plain reverse sweep, written from the chain rule:
 *   A = <phi|psi_L>; lambda = phi; for g = L..1:
 *     psi <- U_g^dagger psi           (psi is now psi_{g-1})
 *     partial_g = <lambda| dU_g |psi>
 *     lambda <- U_g^dagger lambda
 *   grad_g = -2 Re(conj(A) partial_g).
 * psi is overwritten with psi_0 on return.  Writes A to a_out.
 */
int orc_adjoint(cplx *psi, const cplx *phi, int n, const orc_gate *gates, int64_t ng,
                const int32_t *dparam, double *grad, double *a_out) {
    uint64_t N = (uint64_t)1 << n;
    cplx *lam = (cplx *)malloc(sizeof(cplx) * N);
    cplx *tmp = (cplx *)malloc(sizeof(cplx) * N);
    double A[2];
    memcpy(lam, phi, sizeof(cplx) * N);
    orc_inner(phi, psi, n, A);
    if (a_out) {
        a_out[0] = A[0];
        a_out[1] = A[1];
    }
    int rc = 0;
    for (int64_t g = ng - 1; g >= 0; --g) {
        if (orc_apply_gate_inverse(psi, n, &gates[g])) { rc = (int)(g + 1); break; }
        grad[g] = 0.0;
        if (dparam[g] >= 0) {
            double D[8], part[2];
            if (orc_gate_dmatrix(gates[g].kind, gates[g].iarg, gates[g].p, dparam[g], D)) {
                rc = (int)(g + 1);
                break;
            }
            memcpy(tmp, psi, sizeof(cplx) * N);
            orc_apply_ctrl_derivative(tmp, n, gates[g].ctrl, gates[g].target, D);
            orc_inner(lam, tmp, n, part);
            /* Re(conj(A) * part) */
            grad[g] = -2.0 * (A[0] * part[0] + A[1] * part[1]);
        }
        orc_apply_gate_inverse(lam, n, &gates[g]);
    }
    free(lam);
    free(tmp);
    return rc;
}

/* ------------------------------------------------------------ QFT sample --
 * One output of the transform sec. 2.3.2 defines the QFT to be:
 *   beta_x = 2^{-n/2} sum_y omega^{x y} alpha_y,  omega = e^{2 pi i / 2^n}.
 * omega^{xy} depends only on (x y) mod 2^n.  Writing y = yh 2^h + yl with
 * h = ceil(n/2), omega^{xy} = omega^{x yh 2^h} omega^{x yl}; both factors come
 * from tables of e^{2 pi i r / 2^n} built with cos/sin of the exact residue r,
 * so each term costs one complex product.  The sum runs in index order.
 */
void orc_dft_element(const cplx *a, int n, uint64_t x, double *out) {
    uint64_t N = (uint64_t)1 << n, mask = N - 1;
    int h = (n + 1) / 2;
    uint64_t L = (uint64_t)1 << h, H = N >> h;
    cplx *tl = (cplx *)malloc(sizeof(cplx) * L);
    cplx *th = (cplx *)malloc(sizeof(cplx) * H);
    for (uint64_t yl = 0; yl < L; ++yl) {
        uint64_t r = (x * yl) & mask;
        double ang = 2.0 * PI * ldexp((double)r, -n);
        tl[yl] = c_make(cos(ang), sin(ang));
    }
    for (uint64_t yh = 0; yh < H; ++yh) {
        uint64_t r = ((x * yh) << h) & mask;
        double ang = 2.0 * PI * ldexp((double)r, -n);
        th[yh] = c_make(cos(ang), sin(ang));
    }
    cplx s = c_make(0, 0);
    for (uint64_t yh = 0; yh < H; ++yh)
        for (uint64_t yl = 0; yl < L; ++yl) {
            uint64_t y = (yh << h) | yl;
            s = c_add(s, c_mul(c_mul(th[yh], tl[yl]), a[y]));
        }
    double scale = sqrt(ldexp(1.0, -n));
    out[0] = s.re * scale;
    out[1] = s.im * scale;
    free(tl);
    free(th);
}

/* ------------------------------------------------------------ Shor -------
 * sec. 5.1, step 3 with the modular exponentiation done classically: the
 * register pair |0>|a>, a uniform over [0, 2^m) after the HT, becomes
 * |x^a mod N>|a>; measuring the first register with outcome v leaves the
 * second (m qubits) in the equal superposition of every a with
 * x^a mod N = v, each amplitude 1/sqrt(count).  The first register itself is
 * never stored.  x^a mod N by plain square-and-multiply (N < 2^32, so every
 * product fits in 64 bits).  Returns count; count 0 leaves the register zero.
 */
static uint64_t modpow(uint64_t x, uint64_t e, uint64_t N) {
    uint64_t r = 1 % N, b = x % N;
    while (e) {
        if (e & 1) r = (r * b) % N;
        b = (b * b) % N;
        e >>= 1;
    }
    return r;
}

uint64_t orc_modpow(uint64_t x, uint64_t e, uint64_t N) { return modpow(x, e, N); }

uint64_t orc_shor_state(cplx *a, int m, uint64_t N, uint64_t x, uint64_t v) {
    uint64_t M = (uint64_t)1 << m, count = 0;
    for (uint64_t j = 0; j < M; ++j)
        if (modpow(x, j, N) == v) ++count;
    double amp = count ? 1.0 / sqrt((double)count) : 0.0;
    for (uint64_t j = 0; j < M; ++j) a[j] = c_make(modpow(x, j, N) == v ? amp : 0.0, 0.0);
    return count;
}
