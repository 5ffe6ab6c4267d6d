// Element physics shared by the assembly kernels: small FP64 vector algebra,
// the membrane element (St. Venant-Kirchhoff, PSD stress part for the solver
// Jacobian) and the dihedral hinge (paper Sec. 2.5; the readings are listed
// with the oracle's definitions).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace pc {

// ---------------------------------------------------------------- small algebra
struct d3 {
    double x, y, z;
};
__device__ __forceinline__ d3 mk(double a, double b, double c) { return d3{a, b, c}; }
__device__ __forceinline__ d3 operator-(d3 a, d3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ d3 operator+(d3 a, d3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ d3 operator*(double s, d3 a) { return mk(s * a.x, s * a.y, s * a.z); }
__device__ __forceinline__ double dot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ d3 cross(d3 a, d3 b) {
    return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ d3 ld3(const double *p, int i) { return mk(p[3 * i], p[3 * i + 1], p[3 * i + 2]); }

// --------------------------------------------------------------- element physics
// Membrane element (St. Venant-Kirchhoff on the Green strain of the 3x2
// deformation gradient F = sum_k x_k beta_k^T): stress S = 2 mu G + lam tr(G) I.
struct TriShape {
    double b[3][2];  // shape vectors beta_0..2
};

__device__ __forceinline__ void tri_F(const d3 x[3], const TriShape &sh, double F[3][2]) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        F[0][c] = x[0].x * sh.b[0][c] + x[1].x * sh.b[1][c] + x[2].x * sh.b[2][c];
        F[1][c] = x[0].y * sh.b[0][c] + x[1].y * sh.b[1][c] + x[2].y * sh.b[2][c];
        F[2][c] = x[0].z * sh.b[0][c] + x[1].z * sh.b[1][c] + x[2].z * sh.b[2][c];
    }
}

__device__ __forceinline__ void tri_stress(const double F[3][2], double mu, double lam, double S[3]) {
    const double g00 = 0.5 * (F[0][0] * F[0][0] + F[1][0] * F[1][0] + F[2][0] * F[2][0] - 1.0);
    const double g11 = 0.5 * (F[0][1] * F[0][1] + F[1][1] * F[1][1] + F[2][1] * F[2][1] - 1.0);
    const double g01 = 0.5 * (F[0][0] * F[0][1] + F[1][0] * F[1][1] + F[2][0] * F[2][1]);
    const double tr = g00 + g11;
    S[0] = 2.0 * mu * g00 + lam * tr;
    S[1] = 2.0 * mu * g01;
    S[2] = 2.0 * mu * g11 + lam * tr;
}

// Positive part of a symmetric 2x2 matrix [[a, b], [b, c]] (negative
// eigenvalues set to zero).
__device__ __forceinline__ void psd_part(const double S[3], double P[3]) {
    const double a = S[0], b = S[1], c = S[2];
    const double m = 0.5 * (a + c);
    const double r = sqrt(0.25 * (a - c) * (a - c) + b * b);
    const double l1 = m + r, l2 = m - r;
    if (l2 >= 0.0) {
        P[0] = a; P[1] = b; P[2] = c;
        return;
    }
    if (l1 <= 0.0) {
        P[0] = P[1] = P[2] = 0.0;
        return;
    }
    double w0, w1;
    if (fabs(b) > 0.0) {
        w0 = b;
        w1 = l1 - a;
        double nn = sqrt(w0 * w0 + w1 * w1);
        if (!(nn > 0.0)) {
            w0 = l1 - c;
            w1 = b;
            nn = sqrt(w0 * w0 + w1 * w1);
        }
        w0 /= nn;
        w1 /= nn;
    } else if (a >= c) {
        w0 = 1.0; w1 = 0.0;
    } else {
        w0 = 0.0; w1 = 1.0;
    }
    P[0] = l1 * w0 * w0;
    P[1] = l1 * w0 * w1;
    P[2] = l1 * w1 * w1;
}

// Hinge (x0 = a, x1 = b, x2 = c, x3 = d; edge a-b, wings c, d).
// theta = atan2((n1 x n2).e/|e|, n1.n2) with N1 = e x (x2-x0), N2 = (x3-x0) x e.
// Gradient: d/dx2 = -n1/h1, d/dx3 = -n2/h2, d/dx0 = (1-s1) n1/h1 + (1-s2) n2/h2,
// d/dx1 = s1 n1/h1 + s2 n2/h2 (h_k = |N_k|/|e|, s_k = (x_{k+1}-x0).e/|e|^2).
// Returns false when a wing has collapsed (|N_k|^2 < 1e-24 |e|^4).
__device__ __forceinline__ bool hinge_eval(const d3 x[4], double &theta, d3 g[4]) {
    const d3 e = x[1] - x[0], w2 = x[2] - x[0], w3 = x[3] - x[0];
    const d3 N1 = cross(e, w2), N2 = cross(w3, e);
    const double ee = dot(e, e);
    const double q1 = dot(N1, N1), q2 = dot(N2, N2);
    if (!(ee > 0.0) || q1 < 1e-24 * ee * ee || q2 < 1e-24 * ee * ee) return false;
    const double le = sqrt(ee), n1 = sqrt(q1), n2 = sqrt(q2);
    const d3 u1 = (1.0 / n1) * N1, u2 = (1.0 / n2) * N2;
    theta = atan2(dot(cross(u1, u2), e) / le, dot(u1, u2));
    const double h1 = n1 / le, h2 = n2 / le;
    const double s1 = dot(w2, e) / ee, s2 = dot(w3, e) / ee;
    const d3 p1 = (1.0 / h1) * u1, p2 = (1.0 / h2) * u2;
    g[0] = (1.0 - s1) * p1 + (1.0 - s2) * p2;
    g[1] = s1 * p1 + s2 * p2;
    g[2] = (-1.0) * p1;
    g[3] = (-1.0) * p2;
    return true;
}

}  // namespace pc
