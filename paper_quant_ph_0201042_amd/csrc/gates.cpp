// Host-side gate-matrix construction (FP64) and matrix classification.
//
// Operational-error parametrisation of sec. 3.2: a one-qubit gate is the
// rotation U_R(theta) = [[cos t, -sin t], [sin t, cos t]] followed (as a
// right factor) by the phase shift U_P1(phi) = diag(1, e^{i phi}); the
// Hadamard gate is U_R(pi/4) U_P1(pi) and NOT is U_R(pi/2) U_P1(pi), and
// inaccuracies are deviations added to theta and phi.  Unperturbed gates use
// their exact textbook entries so that NOT stays a permutation.
// R_k = diag(1, e^{2 pi i / 2^k}) is the QFT phase gate of sec. 2.3.2.
#include <cmath>
#include <complex>

#include "sv_internal.h"

namespace {

using cd = std::complex<double>;

void store(double U[8], cd a, cd b, cd c, cd d) {
    const cd v[4] = {a, b, c, d};
    for (int i = 0; i < 4; ++i) {
        U[2 * i] = v[i].real();
        U[2 * i + 1] = v[i].imag();
    }
}

// U_R(theta) * U_P1(phi): the phase multiplies the second column.
void rotation_phase(double theta, double phi, double U[8]) {
    const double c = std::cos(theta), s = std::sin(theta);
    const cd e(std::cos(phi), std::sin(phi));
    store(U, cd(c, 0.0), -s * e, cd(s, 0.0), c * e);
}

void phase_shift(double phi, double U[8]) {
    store(U, cd(1.0, 0.0), cd(0.0, 0.0), cd(0.0, 0.0), cd(std::cos(phi), std::sin(phi)));
}

const double kPi = 3.14159265358979323846;

}  // namespace

int svi_gate_matrix(const sv_gate *g, double U[8]) {
    const double *p = g->p;
    switch (g->kind) {
    case SV_G_U:
        for (int i = 0; i < 8; ++i) U[i] = p[i];
        return SV_OK;
    case SV_G_H:
        if (p[0] == 0.0 && p[1] == 0.0) {
            const double h = std::sqrt(0.5);
            store(U, cd(h, 0), cd(h, 0), cd(h, 0), cd(-h, 0));
        } else {
            rotation_phase(kPi / 4 + p[0], kPi + p[1], U);
        }
        return SV_OK;
    case SV_G_X:
        if (p[0] == 0.0 && p[1] == 0.0)
            store(U, cd(0, 0), cd(1, 0), cd(1, 0), cd(0, 0));
        else
            rotation_phase(kPi / 2 + p[0], kPi + p[1], U);
        return SV_OK;
    case SV_G_Y:
        store(U, cd(0, 0), cd(0, -1), cd(0, 1), cd(0, 0));
        return SV_OK;
    case SV_G_Z:
        if (p[1] == 0.0)
            store(U, cd(1, 0), cd(0, 0), cd(0, 0), cd(-1, 0));
        else
            phase_shift(kPi + p[1], U);
        return SV_OK;
    case SV_G_RK:
        if (g->iarg < 0 || g->iarg > 62) return SV_EINVAL;
        phase_shift(2.0 * kPi / std::ldexp(1.0, g->iarg) + p[1], U);
        return SV_OK;
    case SV_G_ROT:
        rotation_phase(p[0], p[1], U);
        return SV_OK;
    case SV_G_SU2: {
        const double r = std::sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2] + p[3] * p[3]);
        if (!(r > 0.0) || !std::isfinite(r)) return SV_EINVAL;
        const double a = p[0] / r, b = p[1] / r, c = p[2] / r, d = p[3] / r;
        store(U, cd(a, b), cd(c, d), cd(-c, d), cd(a, -b));
        return SV_OK;
    }
    default:
        return SV_EINVAL;
    }
}

bool svi_finite(const double U[8]) {
    for (int i = 0; i < 8; ++i)
        if (!std::isfinite(U[i])) return false;
    return true;
}

GateClass svi_classify(const double U[8]) {
    // exact NOT: pure move of amplitudes
    if (U[0] == 0.0 && U[1] == 0.0 && U[2] == 1.0 && U[3] == 0.0 && U[4] == 1.0 && U[5] == 0.0 &&
        U[6] == 0.0 && U[7] == 0.0)
        return GC_PERM;
    // diagonal: only a scaling of each amplitude
    if (U[2] == 0.0 && U[3] == 0.0 && U[4] == 0.0 && U[5] == 0.0) return GC_DIAG;
    return GC_DENSE;
}

extern "C" int sv_gate_matrix(const sv_gate *g, double U[8]) {
    if (!g || !U) return SV_EINVAL;
    if (g->kind == SV_G_SWAP) return SV_EINVAL;
    double tmp[8];
    int rc = svi_gate_matrix(g, tmp);
    if (rc != SV_OK) return rc;
    if (!svi_finite(tmp)) return SV_EINVAL;
    for (int i = 0; i < 8; ++i) U[i] = tmp[i];
    return SV_OK;
}

// Derivative of a gate matrix with respect to one angle deviation:
// which = 0: the rotation angle (p[0] of H, X, ROT), d/dtheta U_R(theta) U_P1(phi)
// = [[-sin, -cos e^{i phi}], [cos, -sin e^{i phi}]]; which = 1: the phase
// angle (p[1] of H, X, ROT, Z, RK), U_R(theta) d/dphi U_P1(phi) with
// d/dphi U_P1(phi) = diag(0, i e^{i phi}).
int svi_gate_dmatrix(const sv_gate *g, int which, double D[8]) {
    double theta = 0.0, phi = 0.0;
    bool rot = true;
    switch (g->kind) {
    case SV_G_H: theta = kPi / 4 + g->p[0]; phi = kPi + g->p[1]; break;
    case SV_G_X: theta = kPi / 2 + g->p[0]; phi = kPi + g->p[1]; break;
    case SV_G_ROT: theta = g->p[0]; phi = g->p[1]; break;
    case SV_G_Z: rot = false; phi = kPi + g->p[1]; break;
    case SV_G_RK:
        if (g->iarg < 0 || g->iarg > 62) return SV_EINVAL;
        rot = false;
        phi = 2.0 * kPi / std::ldexp(1.0, g->iarg) + g->p[1];
        break;
    default: return SV_EINVAL;
    }
    const cd e(std::cos(phi), std::sin(phi));
    const cd ie = cd(0.0, 1.0) * e;
    if (which == 0) {
        if (!rot) return SV_EINVAL;
        const double c = std::cos(theta), s = std::sin(theta);
        store(D, cd(-s, 0), -c * e, cd(c, 0), -s * e);
        return SV_OK;
    }
    if (which == 1) {
        if (rot) {
            const double c = std::cos(theta), s = std::sin(theta);
            store(D, cd(0, 0), -s * ie, cd(0, 0), c * ie);
        } else {
            store(D, cd(0, 0), cd(0, 0), cd(0, 0), ie);
        }
        return SV_OK;
    }
    return SV_EINVAL;
}

extern "C" int sv_gate_dmatrix(const sv_gate *g, int which, double D[8]) {
    if (!g || !D) return SV_EINVAL;
    double tmp[8];
    const int rc = svi_gate_dmatrix(g, which, tmp);
    if (rc != SV_OK) return rc;
    if (!svi_finite(tmp)) return SV_EINVAL;
    for (int i = 0; i < 8; ++i) D[i] = tmp[i];
    return SV_OK;
}
