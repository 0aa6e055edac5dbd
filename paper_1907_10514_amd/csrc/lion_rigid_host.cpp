// Host-side set-up of rigid bodies: body mass, centre of mass, COM velocity,
// angular momentum, principal axes and the body-frame offsets of the members,
// from the ions' positions and velocities.  The principal axes come from a
// cyclic Jacobi eigen-decomposition of the 3x3 inertia tensor.
#include <algorithm>
#include <cmath>
#include <map>

#include "lion_internal.h"

namespace lion {
namespace {

// Principal moments below this fraction of the largest count as zero (a rod of
// point ions has no moment about its axis).
constexpr double kMomentFloor = 1e-10;

// Eigenvalues (ascending) and eigenvectors (columns of E, row-major) of the
// symmetric 3x3 matrix S, by cyclic Jacobi rotations.
void jacobi3(const double S[9], double evals[3], double E[9]) {
    double a[3][3], v[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            a[r][c] = S[3 * r + c];
            v[r][c] = r == c ? 1.0 : 0.0;
        }
    for (int sweep = 0; sweep < 64; ++sweep) {
        const double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
        const double diag = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
        if (off == 0.0 || off <= 1e-34 * diag) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                if (a[p][q] == 0.0) continue;
                const double theta = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                // a <- J^T a J with J the rotation in the (p, q) plane
                for (int k = 0; k < 3; ++k) {
                    const double akp = a[k][p], akq = a[k][q];
                    a[k][p] = c * akp - s * akq;
                    a[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) {
                    const double apk = a[p][k], aqk = a[q][k];
                    a[p][k] = c * apk - s * aqk;
                    a[q][k] = s * apk + c * aqk;
                }
                for (int k = 0; k < 3; ++k) {
                    const double vkp = v[k][p], vkq = v[k][q];
                    v[k][p] = c * vkp - s * vkq;
                    v[k][q] = s * vkp + c * vkq;
                }
            }
    }
    int order[3] = {0, 1, 2};
    std::sort(order, order + 3, [&](int i, int j) { return a[i][i] < a[j][j]; });
    for (int k = 0; k < 3; ++k) {
        evals[k] = a[order[k]][order[k]];
        for (int r = 0; r < 3; ++r) E[3 * r + k] = v[r][order[k]];
    }
}

// Unit quaternion of a rotation matrix (row-major), taking the largest of the
// four candidate square roots for accuracy.
void matrix_quat(const double A[9], double q[4]) {
    const double tr = A[0] + A[4] + A[8];
    double w, x, y, z;
    if (tr > 0.0) {
        const double s = 2.0 * std::sqrt(tr + 1.0);
        w = 0.25 * s;
        x = (A[7] - A[5]) / s;
        y = (A[2] - A[6]) / s;
        z = (A[3] - A[1]) / s;
    } else if (A[0] > A[4] && A[0] > A[8]) {
        const double s = 2.0 * std::sqrt(1.0 + A[0] - A[4] - A[8]);
        w = (A[7] - A[5]) / s;
        x = 0.25 * s;
        y = (A[1] + A[3]) / s;
        z = (A[2] + A[6]) / s;
    } else if (A[4] > A[8]) {
        const double s = 2.0 * std::sqrt(1.0 + A[4] - A[0] - A[8]);
        w = (A[2] - A[6]) / s;
        x = (A[1] + A[3]) / s;
        y = 0.25 * s;
        z = (A[5] + A[7]) / s;
    } else {
        const double s = 2.0 * std::sqrt(1.0 + A[8] - A[0] - A[4]);
        w = (A[3] - A[1]) / s;
        x = (A[2] + A[6]) / s;
        y = (A[5] + A[7]) / s;
        z = 0.25 * s;
    }
    const double nrm = std::sqrt(w * w + x * x + y * y + z * z);
    q[0] = w / nrm;
    q[1] = x / nrm;
    q[2] = y / nrm;
    q[3] = z / nrm;
}

void quat_to_matrix(const double q[4], double A[9]) {
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    A[0] = 1.0 - 2.0 * (y * y + z * z);
    A[1] = 2.0 * (x * y - w * z);
    A[2] = 2.0 * (x * z + w * y);
    A[3] = 2.0 * (x * y + w * z);
    A[4] = 1.0 - 2.0 * (x * x + z * z);
    A[5] = 2.0 * (y * z - w * x);
    A[6] = 2.0 * (x * z - w * y);
    A[7] = 2.0 * (y * z + w * x);
    A[8] = 1.0 - 2.0 * (x * x + y * y);
}

double det3(const double E[9]) {
    return E[0] * (E[4] * E[8] - E[5] * E[7]) - E[1] * (E[3] * E[8] - E[5] * E[6]) +
           E[2] * (E[3] * E[7] - E[4] * E[6]);
}

}  // namespace

int rigid_build(int64_t n, const double* mass, const double* x, const double* y, const double* z,
                const double* vx, const double* vy, const double* vz, const int32_t* body,
                RigidHost& out) {
    std::map<int32_t, int32_t> dense;
    for (int64_t i = 0; i < n; ++i)
        if (body[i] >= 0) dense.emplace(body[i], 0);
    int32_t k = 0;
    for (auto& kv : dense) kv.second = k++;
    const int32_t nb = k;
    out.nbodies = nb;
    out.bodies.assign(nb, RigidDev{});
    out.rb.assign(n, -1);
    out.start.assign(nb + 1, 0);
    out.dbody.assign(3 * n, 0.0);
    out.vx.assign(vx, vx + n);
    out.vy.assign(vy, vy + n);
    out.vz.assign(vz, vz + n);
    for (int64_t i = 0; i < n; ++i)
        if (body[i] >= 0) {
            out.rb[i] = dense[body[i]];
            ++out.start[out.rb[i] + 1];
        }
    for (int32_t b = 0; b < nb; ++b) out.start[b + 1] += out.start[b];
    out.members.assign(out.start[nb], 0);
    std::vector<int32_t> fill(out.start.begin(), out.start.end() - 1);
    for (int64_t i = 0; i < n; ++i)
        if (out.rb[i] >= 0) out.members[fill[out.rb[i]]++] = (int32_t)i;

    for (int32_t b = 0; b < nb; ++b) {
        RigidDev& B = out.bodies[b];
        double M = 0.0, R[3] = {0, 0, 0}, P[3] = {0, 0, 0};
        for (int32_t m = out.start[b]; m < out.start[b + 1]; ++m) {
            const int32_t i = out.members[m];
            M += mass[i];
            R[0] += mass[i] * x[i];
            R[1] += mass[i] * y[i];
            R[2] += mass[i] * z[i];
            P[0] += mass[i] * vx[i];
            P[1] += mass[i] * vy[i];
            P[2] += mass[i] * vz[i];
        }
        if (!(M > 0.0)) return -1;
        for (int c = 0; c < 3; ++c) {
            B.R[c] = R[c] / M;
            B.V[c] = P[c] / M;
        }
        B.M = M;
        double I[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, L[3] = {0, 0, 0};
        for (int32_t m = out.start[b]; m < out.start[b + 1]; ++m) {
            const int32_t i = out.members[m];
            const double d[3] = {x[i] - B.R[0], y[i] - B.R[1], z[i] - B.R[2]};
            const double u[3] = {vx[i] - B.V[0], vy[i] - B.V[1], vz[i] - B.V[2]};
            const double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) I[3 * r + c] += mass[i] * ((r == c ? d2 : 0.0) - d[r] * d[c]);
            L[0] += mass[i] * (d[1] * u[2] - d[2] * u[1]);
            L[1] += mass[i] * (d[2] * u[0] - d[0] * u[2]);
            L[2] += mass[i] * (d[0] * u[1] - d[1] * u[0]);
        }
        double ev[3], E[9];
        jacobi3(I, ev, E);
        if (det3(E) < 0.0)
            for (int r = 0; r < 3; ++r) E[3 * r + 2] = -E[3 * r + 2];
        const double top = std::max(ev[2], 0.0);
        for (int c = 0; c < 3; ++c)
            B.inv_i[c] = (top > 0.0 && ev[c] > kMomentFloor * top) ? 1.0 / ev[c] : 0.0;
        matrix_quat(E, B.q);
        double A[9];
        quat_to_matrix(B.q, A);
        for (int c = 0; c < 3; ++c) B.L[c] = L[c];
        // w = A diag(inv_i) A^T L
        double p[3];
        for (int c = 0; c < 3; ++c) p[c] = (A[c] * L[0] + A[3 + c] * L[1] + A[6 + c] * L[2]) * B.inv_i[c];
        for (int r = 0; r < 3; ++r) B.w[r] = A[3 * r] * p[0] + A[3 * r + 1] * p[1] + A[3 * r + 2] * p[2];
        for (int32_t m = out.start[b]; m < out.start[b + 1]; ++m) {
            const int32_t i = out.members[m];
            const double d[3] = {x[i] - B.R[0], y[i] - B.R[1], z[i] - B.R[2]};
            for (int c = 0; c < 3; ++c)
                out.dbody[c * n + i] = A[c] * d[0] + A[3 + c] * d[1] + A[6 + c] * d[2];
            out.vx[i] = B.V[0] + (B.w[1] * d[2] - B.w[2] * d[1]);
            out.vy[i] = B.V[1] + (B.w[2] * d[0] - B.w[0] * d[2]);
            out.vz[i] = B.V[2] + (B.w[0] * d[1] - B.w[1] * d[0]);
        }
    }
    return 0;
}

}  // namespace lion
