/*
 * FP64 CPU oracle for the implicit cloth step of P-Cloth (Li et al.,
 * arXiv 2008.00409).  TEST INFRASTRUCTURE ONLY: the tests, the smoke check and
 * the benchmark's CPU-baseline leg call it; the product library never does.
 *
 * Plain and slow on purpose: every quantity follows its definition, in double
 * precision, with no blocking, fusion or reordering.  It shares no code with
 * the HIP library.
 *
 * What it computes (paper Sec. 2.5, Eq. 1-3; Sec. 3.2.2 for the matrix):
 *   A  = M - h*df/dv - h^2*df/dx = M + h*(h+beta)*K        (K = -df/dx, PSD)
 *   b  = h*[ f(x + s*h*v) - beta'*K*v ]                    (s = 1, beta' = beta: Eq. 3
 *                                                           as printed; s = 0,
 *                                                           beta' = h+beta: linearised)
 *   solve A dv = b by Jacobi-preconditioned CG;  v += dv;  x += h*v.
 * with K the sum of per-triangle membrane (St. Venant-Kirchhoff) and per-hinge
 * dihedral bending stiffness blocks, gravity as the external force, and pinned
 * vertices eliminated (A_ij = A_ji = 0, A_ii = m_i I, b_i = 0).
 *
 * Layout: positions/velocities are (nv, 3) row-major doubles; triangles (nt, 3)
 * int32; hinges (H, 4) int32 as (a, b, c, d): edge a-b, t1 = (a, b, c) holds the
 * directed edge a->b, t2 = (b, a, d).  Matrices are block-CSR with 3x3 row-major
 * FP64 blocks.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double h, mu, lam, kb, beta;
    double g[3];
    int rhs_mode;   /* 0: b = h f(x + h v) - h beta K v ; 1: b = h f(x) - h (h+beta) K v */
    int hess_mode;  /* 0: PSD solver Jacobian ; 1: exact Hessian (tests only) */
} or_params;

/* ---------------------------------------------------------------- small algebra */
static void sub3(const double *a, const double *b, double *o) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2]; }
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double *a) { return sqrt(dot3(a, a)); }

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------- rest data (tri) */
/* Orthonormal rest frame of a triangle: e1 along X1-X0, n the unit normal,
 * e2 = n x e1.  Dm = [[|X1-X0|, (X2-X0).e1], [0, (X2-X0).e2]], B = Dm^-1 (row
 * major 2x2), A0 = det(Dm)/2.  Returns -1 for a degenerate rest triangle. */
int or_rest_triangle(const double *X0, const double *X1, const double *X2, double *B, double *A0) {
    double E1[3], E2[3], n[3], e1[3], e2[3];
    sub3(X1, X0, E1);
    sub3(X2, X0, E2);
    double l1 = norm3(E1);
    cross3(E1, E2, n);
    double ln = norm3(n);
    if (!(l1 > 0.0) || !(ln > 0.0)) return -1;
    for (int a = 0; a < 3; ++a) { e1[a] = E1[a] / l1; n[a] /= ln; }
    cross3(n, e1, e2);
    double d00 = l1, d01 = dot3(E2, e1), d11 = dot3(E2, e2);
    double det = d00 * d11;
    if (!(det > 0.0)) return -1;
    /* inverse of upper-triangular [[d00, d01], [0, d11]] */
    B[0] = 1.0 / d00;
    B[1] = -d01 / det;
    B[2] = 0.0;
    B[3] = 1.0 / d11;
    *A0 = 0.5 * det;
    return 0;
}

int or_rest_triangles(int nt, const double *X, const int32_t *tris, double *B, double *A0) {
    for (int t = 0; t < nt; ++t) {
        const int32_t *v = tris + 3 * t;
        if (or_rest_triangle(X + 3 * v[0], X + 3 * v[1], X + 3 * v[2], B + 4 * t, A0 + t)) return -1 - t;
    }
    return 0;
}

/* ----------------------------------------------------------------- stretch */
/* Shape vectors: F = sum_k x_k beta_k^T with beta_1 = row 0 of B, beta_2 = row 1,
 * beta_0 = -beta_1 - beta_2 (each in R^2). */
static void shape_vectors(const double *B, double beta[3][2]) {
    beta[1][0] = B[0]; beta[1][1] = B[1];
    beta[2][0] = B[2]; beta[2][1] = B[3];
    beta[0][0] = -B[0] - B[2];
    beta[0][1] = -B[1] - B[3];
}

/* F (3x2, row major F[3*... ]: F[a][c]) from corner positions. */
static void deformation_gradient(const double *x0, const double *x1, const double *x2,
                                 const double beta[3][2], double F[3][2]) {
    const double *xs[3] = {x0, x1, x2};
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 2; ++c) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += xs[k][a] * beta[k][c];
            F[a][c] = s;
        }
}

/* Green strain G = (F^T F - I)/2 and StVK stress S = 2 mu G + lam tr(G) I. */
static void strain_stress(const double F[3][2], double mu, double lam, double G[2][2], double S[2][2]) {
    for (int c = 0; c < 2; ++c)
        for (int d = 0; d < 2; ++d) {
            double s = 0.0;
            for (int a = 0; a < 3; ++a) s += F[a][c] * F[a][d];
            G[c][d] = 0.5 * (s - (c == d ? 1.0 : 0.0));
        }
    double tr = G[0][0] + G[1][1];
    for (int c = 0; c < 2; ++c)
        for (int d = 0; d < 2; ++d) S[c][d] = 2.0 * mu * G[c][d] + (c == d ? lam * tr : 0.0);
}

/* E_t = A0 (mu G:G + lam/2 tr(G)^2) */
double or_stretch_energy(const double *x9, const double *B, double A0, double mu, double lam) {
    double beta[3][2], F[3][2], G[2][2], S[2][2];
    shape_vectors(B, beta);
    deformation_gradient(x9, x9 + 3, x9 + 6, beta, F);
    strain_stress(F, mu, lam, G, S);
    double gg = G[0][0] * G[0][0] + 2.0 * G[0][1] * G[0][1] + G[1][1] * G[1][1];
    double tr = G[0][0] + G[1][1];
    return A0 * (mu * gg + 0.5 * lam * tr * tr);
}

/* f_k = -A0 F S beta_k, f is (3 corners x 3) */
void or_stretch_force(const double *x9, const double *B, double A0, double mu, double lam, double *f) {
    double beta[3][2], F[3][2], G[2][2], S[2][2];
    shape_vectors(B, beta);
    deformation_gradient(x9, x9 + 3, x9 + 6, beta, F);
    strain_stress(F, mu, lam, G, S);
    for (int k = 0; k < 3; ++k) {
        double Sb[2] = {S[0][0] * beta[k][0] + S[0][1] * beta[k][1],
                        S[1][0] * beta[k][0] + S[1][1] * beta[k][1]};
        for (int a = 0; a < 3; ++a) f[3 * k + a] = -A0 * (F[a][0] * Sb[0] + F[a][1] * Sb[1]);
    }
}

/* Clamp negative eigenvalues of a symmetric 2x2 matrix to zero. */
static void psd2(const double S[2][2], double P[2][2]) {
    double a = S[0][0], b = S[0][1], c = S[1][1];
    double m = 0.5 * (a + c);
    double r = sqrt(0.25 * (a - c) * (a - c) + b * b);
    double l1 = m + r, l2 = m - r;
    if (l2 >= 0.0) { memcpy(P, S, sizeof(double) * 4); return; }
    if (l1 <= 0.0) { memset(P, 0, sizeof(double) * 4); return; }
    /* only l1 > 0 survives: P = l1 w w^T, w the unit eigenvector of l1 */
    double w0, w1;
    if (fabs(b) > 0.0) {
        w0 = b; w1 = l1 - a;
        double nn = sqrt(w0 * w0 + w1 * w1);
        if (!(nn > 0.0)) { w0 = l1 - c; w1 = b; nn = sqrt(w0 * w0 + w1 * w1); }
        w0 /= nn; w1 /= nn;
    } else if (a >= c) { w0 = 1.0; w1 = 0.0; }
    else { w0 = 0.0; w1 = 1.0; }
    P[0][0] = l1 * w0 * w0; P[0][1] = l1 * w0 * w1;
    P[1][0] = l1 * w1 * w0; P[1][1] = l1 * w1 * w1;
}

/* K_kl = A0 [ mu (b_k.b_l) F F^T + mu u_l u_k^T + lam u_k u_l^T + (b_k^T S b_l) I ],
 * u_k = F b_k; in the solver mode (exact = 0) S is replaced by its PSD part in the
 * last term only.  K is 9x9 row major: K[(3k+a)*9 + 3l+b] = d2E / dx_k[a] dx_l[b]. */
void or_stretch_K(const double *x9, const double *B, double A0, double mu, double lam, int exact, double *K) {
    double beta[3][2], F[3][2], G[2][2], S[2][2], Sp[2][2];
    shape_vectors(B, beta);
    deformation_gradient(x9, x9 + 3, x9 + 6, beta, F);
    strain_stress(F, mu, lam, G, S);
    if (exact) memcpy(Sp, S, sizeof(Sp)); else psd2(S, Sp);
    double u[3][3], FFt[3][3];
    for (int k = 0; k < 3; ++k)
        for (int a = 0; a < 3; ++a) u[k][a] = F[a][0] * beta[k][0] + F[a][1] * beta[k][1];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) FFt[a][b] = F[a][0] * F[b][0] + F[a][1] * F[b][1];
    for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) {
            double bb = beta[k][0] * beta[l][0] + beta[k][1] * beta[l][1];
            double bSb = 0.0;
            for (int c = 0; c < 2; ++c)
                for (int d = 0; d < 2; ++d) bSb += beta[k][c] * Sp[c][d] * beta[l][d];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    double v = mu * bb * FFt[a][b] + mu * u[l][a] * u[k][b] + lam * u[k][a] * u[l][b];
                    if (a == b) v += bSb;
                    K[(3 * k + a) * 9 + 3 * l + b] = A0 * v;
                }
        }
}

/* ----------------------------------------------------------------- bending */
/* Dihedral angle of hinge (x0 = a, x1 = b, x2 = c, x3 = d):
 * e = x1 - x0, N1 = e x (x2 - x0), N2 = (x3 - x0) x e,
 * theta = atan2((n1 x n2).e/|e|, n1.n2). */
double or_hinge_angle(const double *x12) {
    const double *x0 = x12, *x1 = x12 + 3, *x2 = x12 + 6, *x3 = x12 + 9;
    double e[3], w2[3], w3[3], N1[3], N2[3], c[3];
    sub3(x1, x0, e);
    sub3(x2, x0, w2);
    sub3(x3, x0, w3);
    cross3(e, w2, N1);
    cross3(w3, e, N2);
    double n1 = norm3(N1), n2 = norm3(N2), le = norm3(e);
    double u1[3] = {N1[0] / n1, N1[1] / n1, N1[2] / n1};
    double u2[3] = {N2[0] / n2, N2[1] / n2, N2[2] / n2};
    cross3(u1, u2, c);
    return atan2(dot3(c, e) / le, dot3(u1, u2));
}

/* 1 if the hinge is too degenerate to contribute (a wing triangle has collapsed). */
static int hinge_degenerate(const double *x12) {
    const double *x0 = x12, *x1 = x12 + 3, *x2 = x12 + 6, *x3 = x12 + 9;
    double e[3], w2[3], w3[3], N1[3], N2[3];
    sub3(x1, x0, e);
    sub3(x2, x0, w2);
    sub3(x3, x0, w3);
    cross3(e, w2, N1);
    cross3(w3, e, N2);
    double ee = dot3(e, e);
    return !(ee > 0.0) || dot3(N1, N1) < 1e-24 * ee * ee || dot3(N2, N2) < 1e-24 * ee * ee;
}

/* Gradient of theta (12 values, corner-major):
 *   d/dx2 = -n1/h1, d/dx3 = -n2/h2,
 *   d/dx0 = (1-s1) n1/h1 + (1-s2) n2/h2,  d/dx1 = s1 n1/h1 + s2 n2/h2,
 * with h_k = |N_k|/|e| and s_k = (x_{k+1} - x0).e/|e|^2. */
void or_hinge_grad(const double *x12, double *g) {
    const double *x0 = x12, *x1 = x12 + 3, *x2 = x12 + 6, *x3 = x12 + 9;
    double e[3], w2[3], w3[3], N1[3], N2[3];
    sub3(x1, x0, e);
    sub3(x2, x0, w2);
    sub3(x3, x0, w3);
    cross3(e, w2, N1);
    cross3(w3, e, N2);
    double ee = dot3(e, e), le = sqrt(ee);
    double n1 = norm3(N1), n2 = norm3(N2);
    double h1 = n1 / le, h2 = n2 / le;
    double s1 = dot3(w2, e) / ee, s2 = dot3(w3, e) / ee;
    for (int a = 0; a < 3; ++a) {
        double p1 = N1[a] / n1 / h1, p2 = N2[a] / n2 / h2;
        g[0 + a] = (1.0 - s1) * p1 + (1.0 - s2) * p2;
        g[3 + a] = s1 * p1 + s2 * p2;
        g[6 + a] = -p1;
        g[9 + a] = -p2;
    }
}

/* E_h = kb ch (theta - theta_bar)^2 */
double or_bend_energy(const double *x12, double ch, double tbar, double kb) {
    if (hinge_degenerate(x12)) return 0.0;
    double d = or_hinge_angle(x12) - tbar;
    return kb * ch * d * d;
}

/* f = -2 kb ch (theta - theta_bar) grad theta */
void or_bend_force(const double *x12, double ch, double tbar, double kb, double *f) {
    if (hinge_degenerate(x12)) { memset(f, 0, 12 * sizeof(double)); return; }
    double g[12];
    or_hinge_grad(x12, g);
    double s = -2.0 * kb * ch * (or_hinge_angle(x12) - tbar);
    for (int i = 0; i < 12; ++i) f[i] = s * g[i];
}

/* Solver mode: K = 2 kb ch grad grad^T (Gauss-Newton).  Exact mode adds
 * 2 kb ch (theta - theta_bar) Hess(theta), the Hessian taken as the central
 * difference of the analytic gradient (step 1e-6 |e|), symmetrised.
 * K is 12x12 row major. */
void or_bend_K(const double *x12, double ch, double tbar, double kb, int exact, double *K) {
    if (hinge_degenerate(x12)) { memset(K, 0, 144 * sizeof(double)); return; }
    double g[12];
    or_hinge_grad(x12, g);
    double c = 2.0 * kb * ch;
    for (int i = 0; i < 12; ++i)
        for (int j = 0; j < 12; ++j) K[i * 12 + j] = c * g[i] * g[j];
    if (!exact) return;
    double e[3];
    sub3(x12 + 3, x12, e);
    double step = 1e-6 * norm3(e);
    double th = or_hinge_angle(x12) - tbar;
    double Hs[144];
    for (int j = 0; j < 12; ++j) {
        double xp[12], xm[12], gp[12], gm[12];
        memcpy(xp, x12, sizeof(xp));
        memcpy(xm, x12, sizeof(xm));
        xp[j] += step;
        xm[j] -= step;
        or_hinge_grad(xp, gp);
        or_hinge_grad(xm, gm);
        for (int i = 0; i < 12; ++i) Hs[i * 12 + j] = (gp[i] - gm[i]) / (2.0 * step);
    }
    for (int i = 0; i < 12; ++i)
        for (int j = 0; j < 12; ++j) K[i * 12 + j] += c * th * 0.5 * (Hs[i * 12 + j] + Hs[j * 12 + i]);
}

/* ------------------------------------------------------------------ contact */
/* Proximity (repulsion) element between 4 vertices: a vertex-face pair
 * (p; a, b, c) with c = (1, -w_a, -w_b, -w_c) from the closest point's
 * barycentric weights, or an edge-edge pair (a, b; c, d) with
 * c = (1 - s, s, -(1 - t), -t) from the closest points' parameters.  The
 * weights (which sum to zero) and the unit normal n come with the pair from
 * the proximity query and are constants of the step.  Gap g = n . sum_k c_k x_k;
 * energy kc/2 (eta - g)^2 while g < eta (eta: thickness), zero otherwise. */
static double contact_gap(const double *x12, const double *c, const double *n) {
    double s[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < 4; ++k)
        for (int a = 0; a < 3; ++a) s[a] += c[k] * x12[3 * k + a];
    return dot3(n, s);
}

double or_contact_energy(const double *x12, const double *c, const double *n, double eta, double kc) {
    double g = contact_gap(x12, c, n);
    return g < eta ? 0.5 * kc * (eta - g) * (eta - g) : 0.0;
}

/* f_k = -dE/dx_k = kc (eta - g) c_k n while g < eta. */
void or_contact_force(const double *x12, const double *c, const double *n, double eta, double kc, double *f12) {
    double g = contact_gap(x12, c, n);
    double m = g < eta ? kc * (eta - g) : 0.0;
    for (int k = 0; k < 4; ++k)
        for (int a = 0; a < 3; ++a) f12[3 * k + a] = m * c[k] * n[a];
}

/* K = d2E/dx2 (12 x 12, row major): blocks kc c_k c_l n n^T while g < eta
 * (g is linear in x, so this is the exact Hessian and it is PSD). */
void or_contact_K(const double *x12, const double *c, const double *n, double eta, double kc, double *K) {
    double g = contact_gap(x12, c, n);
    for (int i = 0; i < 144; ++i) K[i] = 0.0;
    if (!(g < eta)) return;
    for (int k = 0; k < 4; ++k)
        for (int l = 0; l < 4; ++l)
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) K[(3 * k + a) * 12 + 3 * l + b] = kc * c[k] * c[l] * n[a] * n[b];
}

/* ------------------------------------------------------------------ topology */
typedef struct { int64_t key; int32_t tri; int32_t corner; } dir_edge;

static int cmp_dir_edge(const void *pa, const void *pb) {
    const dir_edge *a = (const dir_edge *)pa, *b = (const dir_edge *)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->tri != b->tri) return a->tri < b->tri ? -1 : 1;
    return a->corner - b->corner;
}

/* Interior edges become hinges, listed in ascending (min, max) vertex order.
 * t1 is the lower-numbered of the two triangles; (a, b) is its directed edge,
 * c its third vertex; d is the third vertex of the other triangle, which must
 * hold b->a.  Returns H, -1 for an edge in more than two triangles, -2 for an
 * inconsistently oriented pair, -3 if cap is too small. */
int or_build_hinges(int nv, int nt, const int32_t *tris, int32_t *hinges, int cap) {
    dir_edge *E = (dir_edge *)malloc(sizeof(dir_edge) * (size_t)3 * nt);
    for (int t = 0; t < nt; ++t)
        for (int k = 0; k < 3; ++k) {
            int64_t p = tris[3 * t + k], q = tris[3 * t + (k + 1) % 3];
            int64_t lo = p < q ? p : q, hi = p < q ? q : p;
            E[3 * t + k].key = lo * (int64_t)nv + hi;
            E[3 * t + k].tri = t;
            E[3 * t + k].corner = k;
        }
    qsort(E, (size_t)3 * nt, sizeof(dir_edge), cmp_dir_edge);
    int H = 0;
    size_t i = 0, n = (size_t)3 * nt;
    int status = 0;
    while (i < n) {
        size_t j = i + 1;
        while (j < n && E[j].key == E[i].key) ++j;
        if (j - i > 2) { status = -1; break; }
        if (j - i == 2) {
            const dir_edge *e1 = &E[i], *e2 = &E[i + 1];  /* e1->tri < e2->tri */
            int a = tris[3 * e1->tri + e1->corner], b = tris[3 * e1->tri + (e1->corner + 1) % 3];
            int c = tris[3 * e1->tri + (e1->corner + 2) % 3];
            int p = tris[3 * e2->tri + e2->corner], q = tris[3 * e2->tri + (e2->corner + 1) % 3];
            int d = tris[3 * e2->tri + (e2->corner + 2) % 3];
            if (!(p == b && q == a)) { status = -2; break; }
            if (H >= cap) { status = -3; break; }
            hinges[4 * H + 0] = a;
            hinges[4 * H + 1] = b;
            hinges[4 * H + 2] = c;
            hinges[4 * H + 3] = d;
            ++H;
        }
        i = j;
    }
    free(E);
    return status ? status : H;
}

/* c_h = 3 |e|^2 / (A1 + A2) from rest positions; theta_bar = rest dihedral angle. */
void or_rest_hinges(const double *X, int H, const int32_t *hinges, double *ch, double *tbar) {
    for (int h = 0; h < H; ++h) {
        double x12[12];
        for (int k = 0; k < 4; ++k) memcpy(x12 + 3 * k, X + 3 * hinges[4 * h + k], 3 * sizeof(double));
        double e[3], w2[3], w3[3], N1[3], N2[3];
        sub3(x12 + 3, x12, e);
        sub3(x12 + 6, x12, w2);
        sub3(x12 + 9, x12, w3);
        cross3(e, w2, N1);
        cross3(w3, e, N2);
        double A1 = 0.5 * norm3(N1), A2 = 0.5 * norm3(N2);
        ch[h] = 3.0 * dot3(e, e) / (A1 + A2);
        tbar[h] = or_hinge_angle(x12);
    }
}

/* ------------------------------------------------------------------- pattern */
static int cmp_i64(const void *pa, const void *pb) {
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    return a < b ? -1 : (a > b ? 1 : 0);
}

/* Block pattern: every (row, col) pair of vertices that share an element
 * (triangle, hinge or contact; the diagonal included), sorted and
 * de-duplicated.  Returns nnzb (or -1 if cap is
 * too small); rowptr has nv+1 entries. */
int or_pattern2(int nv, int nt, const int32_t *tris, int H, const int32_t *hinges, int nc, const int32_t *cverts,
                int32_t *rowptr, int32_t *colidx, int cap) {
    size_t nkeys = (size_t)9 * nt + (size_t)16 * H + (size_t)16 * nc + (size_t)nv;
    int64_t *keys = (int64_t *)malloc(sizeof(int64_t) * (nkeys ? nkeys : 1));
    size_t m = 0;
    /* M is diagonal with positive masses (Eq. 3): every row holds its
       diagonal block, also a vertex that no element touches */
    for (int i = 0; i < nv; ++i) keys[m++] = (int64_t)i * nv + i;
    for (int t = 0; t < nt; ++t)
        for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l) keys[m++] = (int64_t)tris[3 * t + k] * nv + tris[3 * t + l];
    for (int h = 0; h < H; ++h)
        for (int k = 0; k < 4; ++k)
            for (int l = 0; l < 4; ++l) keys[m++] = (int64_t)hinges[4 * h + k] * nv + hinges[4 * h + l];
    for (int e = 0; e < nc; ++e)
        for (int k = 0; k < 4; ++k)
            for (int l = 0; l < 4; ++l) keys[m++] = (int64_t)cverts[4 * e + k] * nv + cverts[4 * e + l];
    qsort(keys, nkeys, sizeof(int64_t), cmp_i64);
    int nnzb = 0;
    for (int r = 0; r <= nv; ++r) rowptr[r] = 0;
    for (size_t i = 0; i < nkeys; ++i) {
        if (i > 0 && keys[i] == keys[i - 1]) continue;
        if (nnzb >= cap) { free(keys); return -1; }
        int row = (int)(keys[i] / nv), col = (int)(keys[i] % nv);
        colidx[nnzb++] = col;
        rowptr[row + 1]++;
    }
    for (int r = 0; r < nv; ++r) rowptr[r + 1] += rowptr[r];
    free(keys);
    return nnzb;
}

int or_pattern(int nv, int nt, const int32_t *tris, int H, const int32_t *hinges,
               int32_t *rowptr, int32_t *colidx, int cap) {
    return or_pattern2(nv, nt, tris, H, hinges, 0, NULL, rowptr, colidx, cap);
}

static int find_block(const int32_t *rowptr, const int32_t *colidx, int row, int col) {
    int lo = rowptr[row], hi = rowptr[row + 1] - 1;
    while (lo <= hi) {
        int mid = (lo + hi) / 2;
        if (colidx[mid] == col) return mid;
        if (colidx[mid] < col) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* ------------------------------------------------------------------ assembly */
typedef struct {
    int nc;
    const int32_t *verts;    /* nc x 4 */
    const double *w;         /* nc x 4 weights c_k (sum zero) */
    const double *n;         /* nc x 3 unit normals */
    double eta, kc;          /* thickness, stiffness */
} or_contacts;
/* Internal + gravity force at positions y (nv x 3). */
static void total_force(int nv, int nt, const int32_t *tris, const double *Bt, const double *A0,
                        int H, const int32_t *hinges, const double *ch, const double *tbar,
                        const or_contacts *C, const double *mass, const or_params *P, const double *y,
                        double *f) {
    for (int i = 0; i < nv; ++i)
        for (int a = 0; a < 3; ++a) f[3 * i + a] = mass[i] * P->g[a];
    double *ft = (double *)malloc(sizeof(double) * 9 * (size_t)nt);
    double *fh = (double *)malloc(sizeof(double) * 12 * (size_t)H);
#pragma omp parallel for schedule(static)
    for (int t = 0; t < nt; ++t) {
        double x9[9];
        for (int k = 0; k < 3; ++k) memcpy(x9 + 3 * k, y + 3 * tris[3 * t + k], 3 * sizeof(double));
        or_stretch_force(x9, Bt + 4 * t, A0[t], P->mu, P->lam, ft + 9 * t);
    }
#pragma omp parallel for schedule(static)
    for (int h = 0; h < H; ++h) {
        double x12[12];
        for (int k = 0; k < 4; ++k) memcpy(x12 + 3 * k, y + 3 * hinges[4 * h + k], 3 * sizeof(double));
        or_bend_force(x12, ch[h], tbar[h], P->kb, fh + 12 * h);
    }
    for (int t = 0; t < nt; ++t)
        for (int k = 0; k < 3; ++k)
            for (int a = 0; a < 3; ++a) f[3 * tris[3 * t + k] + a] += ft[9 * t + 3 * k + a];
    for (int h = 0; h < H; ++h)
        for (int k = 0; k < 4; ++k)
            for (int a = 0; a < 3; ++a) f[3 * hinges[4 * h + k] + a] += fh[12 * h + 3 * k + a];
    for (int e = 0; e < C->nc; ++e) {
        double x12[12], fc[12];
        for (int k = 0; k < 4; ++k) memcpy(x12 + 3 * k, y + 3 * C->verts[4 * e + k], 3 * sizeof(double));
        or_contact_force(x12, C->w + 4 * e, C->n + 3 * e, C->eta, C->kc, fc);
        for (int k = 0; k < 4; ++k)
            for (int a = 0; a < 3; ++a) f[3 * C->verts[4 * e + k] + a] += fc[3 * k + a];
    }
    free(ft);
    free(fh);
}

/* Stiffness K = sum of element blocks at positions x, accumulated into the
 * pattern (vals: nnzb x 9, zeroed here), in element order (triangles, then
 * hinges).  Returns -1 if a block is missing from the pattern. */
static int stiffness(int nv, int nt, const int32_t *tris, const double *Bt, const double *A0,
                     int H, const int32_t *hinges, const double *ch, const double *tbar,
                     const or_contacts *C, const or_params *P, const double *x, const int32_t *rowptr,
                     const int32_t *colidx, double *vals) {
    int nnzb = rowptr[nv];
    memset(vals, 0, sizeof(double) * 9 * (size_t)nnzb);
    double *Kt = (double *)malloc(sizeof(double) * 81 * (size_t)nt);
    double *Kh = (double *)malloc(sizeof(double) * 144 * (size_t)H);
#pragma omp parallel for schedule(static)
    for (int t = 0; t < nt; ++t) {
        double x9[9];
        for (int k = 0; k < 3; ++k) memcpy(x9 + 3 * k, x + 3 * tris[3 * t + k], 3 * sizeof(double));
        or_stretch_K(x9, Bt + 4 * t, A0[t], P->mu, P->lam, P->hess_mode, Kt + 81 * t);
    }
#pragma omp parallel for schedule(static)
    for (int h = 0; h < H; ++h) {
        double x12[12];
        for (int k = 0; k < 4; ++k) memcpy(x12 + 3 * k, x + 3 * hinges[4 * h + k], 3 * sizeof(double));
        or_bend_K(x12, ch[h], tbar[h], P->kb, P->hess_mode, Kh + 144 * h);
    }
    int status = 0;
    for (int t = 0; t < nt && !status; ++t)
        for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l) {
                int s = find_block(rowptr, colidx, tris[3 * t + k], tris[3 * t + l]);
                if (s < 0) { status = -1; break; }
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) vals[9 * s + 3 * a + b] += Kt[81 * t + (3 * k + a) * 9 + 3 * l + b];
            }
    for (int h = 0; h < H && !status; ++h)
        for (int k = 0; k < 4; ++k)
            for (int l = 0; l < 4; ++l) {
                int s = find_block(rowptr, colidx, hinges[4 * h + k], hinges[4 * h + l]);
                if (s < 0) { status = -1; break; }
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) vals[9 * s + 3 * a + b] += Kh[144 * h + (3 * k + a) * 12 + 3 * l + b];
            }
    for (int e = 0; e < C->nc && !status; ++e) {
        double x12[12], Kc[144];
        for (int k = 0; k < 4; ++k) memcpy(x12 + 3 * k, x + 3 * C->verts[4 * e + k], 3 * sizeof(double));
        or_contact_K(x12, C->w + 4 * e, C->n + 3 * e, C->eta, C->kc, Kc);
        for (int k = 0; k < 4 && !status; ++k)
            for (int l = 0; l < 4; ++l) {
                int s = find_block(rowptr, colidx, C->verts[4 * e + k], C->verts[4 * e + l]);
                if (s < 0) { status = -1; break; }
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) vals[9 * s + 3 * a + b] += Kc[(3 * k + a) * 12 + 3 * l + b];
            }
    }
    free(Kt);
    free(Kh);
    return status;
}

/* y = K x over the pattern (plain block-CSR product). */
static void block_spmv(int nv, const int32_t *rowptr, const int32_t *colidx, const double *vals,
                       const double *x, double *y) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nv; ++i) {
        double s[3] = {0.0, 0.0, 0.0};
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            const double *blk = vals + 9 * (size_t)p;
            const double *xj = x + 3 * colidx[p];
            for (int a = 0; a < 3; ++a) s[a] += blk[3 * a] * xj[0] + blk[3 * a + 1] * xj[1] + blk[3 * a + 2] * xj[2];
        }
        for (int a = 0; a < 3; ++a) y[3 * i + a] = s[a];
    }
}

/* Assemble A (vals: nnzb x 9 on the given pattern), b (nv x 3), the Jacobi
 * diagonal diag(A) (nv x 3) and the pinned-neighbour remainder
 * D_i = -h(h+beta) sum_{j pinned, j != i} K_ij for unpinned i, 0 for pinned i
 * (nv x 9), from state (x, v).  Returns 0, or -1 on a pattern mismatch. */
int or_assemble2(int nv, int nt, const int32_t *tris, const double *Bt, const double *A0,
                 int H, const int32_t *hinges, const double *ch, const double *tbar,
                 int nc, const int32_t *cverts, const double *cw, const double *cn, double eta, double kc,
                 const double *mass, const uint8_t *pinned, const or_params *P,
                 const double *x, const double *v, const int32_t *rowptr, const int32_t *colidx,
                 double *vals, double *b, double *diag, double *D) {
    int nnzb = rowptr[nv];
    or_contacts C0 = {nc, cverts, cw, cn, eta, kc};
    const or_contacts *C = &C0;
    if (stiffness(nv, nt, tris, Bt, A0, H, hinges, ch, tbar, C, P, x, rowptr, colidx, vals)) return -1;
    /* right-hand side */
    double s = P->rhs_mode == 0 ? 1.0 : 0.0;
    double bk = P->rhs_mode == 0 ? P->beta : P->h + P->beta;
    double *y = (double *)malloc(sizeof(double) * 3 * (size_t)nv);
    double *f = (double *)malloc(sizeof(double) * 3 * (size_t)nv);
    double *Kv = (double *)malloc(sizeof(double) * 3 * (size_t)nv);
    for (int i = 0; i < 3 * nv; ++i) y[i] = x[i] + s * P->h * v[i];
    total_force(nv, nt, tris, Bt, A0, H, hinges, ch, tbar, C, mass, P, y, f);
    block_spmv(nv, rowptr, colidx, vals, v, Kv);
    for (int i = 0; i < nv; ++i)
        for (int a = 0; a < 3; ++a)
            b[3 * i + a] = pinned[i] ? 0.0 : P->h * (f[3 * i + a] - bk * Kv[3 * i + a]);
    /* remainder D from the stiffness before elimination */
    double c = P->h * (P->h + P->beta);
    for (int i = 0; i < nv; ++i) {
        double *Di = D + 9 * (size_t)i;
        memset(Di, 0, 9 * sizeof(double));
        if (pinned[i]) continue;
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int j = colidx[p];
            if (j == i || !pinned[j]) continue;
            for (int q = 0; q < 9; ++q) Di[q] -= c * vals[9 * (size_t)p + q];
        }
    }
    /* A = M + c K, then Dirichlet elimination */
    for (int i = 0; i < nv; ++i)
        for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            int j = colidx[p];
            double *blk = vals + 9 * (size_t)p;
            if (pinned[i] || pinned[j]) {
                for (int q = 0; q < 9; ++q) blk[q] = 0.0;
                if (i == j) blk[0] = blk[4] = blk[8] = mass[i];
                continue;
            }
            for (int q = 0; q < 9; ++q) blk[q] *= c;
            if (i == j) { blk[0] += mass[i]; blk[4] += mass[i]; blk[8] += mass[i]; }
        }
    for (int i = 0; i < nv; ++i) {
        int p = find_block(rowptr, colidx, i, i);
        for (int a = 0; a < 3; ++a) diag[3 * i + a] = vals[9 * (size_t)p + 4 * a];
    }
    (void)nnzb;
    free(y);
    free(f);
    free(Kv);
    return 0;
}

int or_assemble(int nv, int nt, const int32_t *tris, const double *Bt, const double *A0,
                int H, const int32_t *hinges, const double *ch, const double *tbar,
                const double *mass, const uint8_t *pinned, const or_params *P,
                const double *x, const double *v, const int32_t *rowptr, const int32_t *colidx,
                double *vals, double *b, double *diag, double *D) {
    return or_assemble2(nv, nt, tris, Bt, A0, H, hinges, ch, tbar, 0, NULL, NULL, NULL, 0.0, 0.0, mass, pinned, P,
                        x, v, rowptr, colidx, vals, b, diag, D);
}

/* y = A x on an assembled block-CSR matrix. */
void or_spmv(int nv, const int32_t *rowptr, const int32_t *colidx, const double *vals,
             const double *x, double *y) {
    block_spmv(nv, rowptr, colidx, vals, x, y);
}

static double dotn(int n, const double *a, const double *b) {
    double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (int i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Solve the 3x3 system M z = r by Gaussian elimination with partial pivoting
 * (M row-major, left unchanged). */
static void solve3(const double *M, const double *r, double *z) {
    double a[3][4];
    for (int i = 0; i < 3; ++i) {
        for (int j = 0; j < 3; ++j) a[i][j] = M[3 * i + j];
        a[i][3] = r[i];
    }
    for (int k = 0; k < 3; ++k) {
        int piv = k;
        for (int i = k + 1; i < 3; ++i)
            if (fabs(a[i][k]) > fabs(a[piv][k])) piv = i;
        if (piv != k)
            for (int j = 0; j < 4; ++j) { double t = a[k][j]; a[k][j] = a[piv][j]; a[piv][j] = t; }
        for (int i = k + 1; i < 3; ++i) {
            double f = a[i][k] / a[k][k];
            for (int j = k; j < 4; ++j) a[i][j] -= f * a[k][j];
        }
    }
    for (int i = 2; i >= 0; --i) {
        double s = a[i][3];
        for (int j = i + 1; j < 3; ++j) s -= a[i][j] * z[j];
        z[i] = s / a[i][i];
    }
}

/* Preconditioner application z = P^-1 r: precond 0 is Jacobi (P = diag(A)),
 * precond 1 is block Jacobi (P = the 3x3 diagonal blocks A_ii). */
static void apply_precond(int nv, const int32_t *rowptr, const int32_t *colidx, const double *vals,
                          const double *diag, int precond, const double *r, double *z) {
    if (precond == 0) {
        for (int i = 0; i < 3 * nv; ++i) z[i] = r[i] / diag[i];
        return;
    }
    for (int i = 0; i < nv; ++i) {
        int p = find_block(rowptr, colidx, i, i);
        solve3(vals + 9 * (size_t)p, r + 3 * i, z + 3 * i);
    }
}

/* Preconditioned CG on A x = b from the initial guess in x (paper Sec. 2.5;
 * preconditioner as in apply_precond).  Stops when ||r_k|| <= tol ||b||
 * (recursive residual) or after maxit iterations.  b = 0 gives x = 0 and no
 * iterations.  Returns 0 if converged, 1 if not.  out[0] = iterations,
 * out[1] = recursive relative residual, out[2] = true relative residual
 * ||b - A x|| / ||b|| at exit. */
int or_pcg2(int nv, const int32_t *rowptr, const int32_t *colidx, const double *vals,
            const double *b, const double *diag, double *x, double tol, int maxit, int precond, double *out) {
    int n = 3 * nv;
    double bnorm = sqrt(dotn(n, b, b));
    if (bnorm == 0.0) {
        memset(x, 0, sizeof(double) * n);
        out[0] = 0; out[1] = 0.0; out[2] = 0.0;
        return 0;
    }
    double *r = (double *)malloc(sizeof(double) * n);
    double *z = (double *)malloc(sizeof(double) * n);
    double *p = (double *)malloc(sizeof(double) * n);
    double *q = (double *)malloc(sizeof(double) * n);
    block_spmv(nv, rowptr, colidx, vals, x, q);
    for (int i = 0; i < n; ++i) r[i] = b[i] - q[i];
    apply_precond(nv, rowptr, colidx, vals, diag, precond, r, z);
    memcpy(p, z, sizeof(double) * n);
    double rz = dotn(n, r, z);
    double rr = dotn(n, r, r);
    int it = 0;
    while (sqrt(rr) > tol * bnorm && it < maxit) {
        block_spmv(nv, rowptr, colidx, vals, p, q);
        double alpha = rz / dotn(n, p, q);
        for (int i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
        apply_precond(nv, rowptr, colidx, vals, diag, precond, r, z);
        double rz_new = dotn(n, r, z);
        rr = dotn(n, r, r);
        double beta = rz_new / rz;
        rz = rz_new;
        for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        ++it;
    }
    block_spmv(nv, rowptr, colidx, vals, x, q);
    double tr = 0.0;
    for (int i = 0; i < n; ++i) tr += (b[i] - q[i]) * (b[i] - q[i]);
    out[0] = it;
    out[1] = sqrt(rr) / bnorm;
    out[2] = sqrt(tr) / bnorm;
    free(r); free(z); free(p); free(q);
    return sqrt(rr) <= tol * bnorm ? 0 : 1;
}

/* Preconditioned CG in the single-reduction form of Chronopoulos and Gear
 * ("s-step iterative methods for symmetric linear systems", 1989, the s = 1
 * case).  Each iteration takes one product w = A u of the preconditioned
 * residual u = P^-1 r and the two dots gamma = r.u and delta = w.u together;
 * the direction p and s = A p follow from recurrences:
 *   beta_k  = gamma_k / gamma_{k-1}                 (beta_0 = 0)
 *   alpha_k = gamma_k / (delta_k - beta_k gamma_k / alpha_{k-1})
 *   p_k = u_k + beta_k p_{k-1},   s_k = w_k + beta_k s_{k-1}
 *   x_{k+1} = x_k + alpha_k p_k,  r_{k+1} = r_k - alpha_k s_k.
 * In exact arithmetic the iterates are those of or_pcg2 (alpha_k, beta_k
 * are the same numbers: delta_k - beta_k gamma_k / alpha_{k-1} = p_k.A p_k).
 * Same preconditioners, stopping rule, outputs and return value as or_pcg2;
 * out[3] = 1 if a denominator was not positive (breakdown), else 0. */
int or_pcg_cg(int nv, const int32_t *rowptr, const int32_t *colidx, const double *vals,
              const double *b, const double *diag, double *x, double tol, int maxit, int precond, double *out) {
    int n = 3 * nv;
    double bnorm = sqrt(dotn(n, b, b));
    out[3] = 0.0;
    if (bnorm == 0.0) {
        memset(x, 0, sizeof(double) * n);
        out[0] = 0; out[1] = 0.0; out[2] = 0.0;
        return 0;
    }
    double *r = (double *)malloc(sizeof(double) * n);
    double *u = (double *)malloc(sizeof(double) * n);
    double *w = (double *)malloc(sizeof(double) * n);
    double *p = (double *)calloc(n, sizeof(double));
    double *s = (double *)calloc(n, sizeof(double));
    block_spmv(nv, rowptr, colidx, vals, x, w);
    for (int i = 0; i < n; ++i) r[i] = b[i] - w[i];
    apply_precond(nv, rowptr, colidx, vals, diag, precond, r, u);
    double rr = dotn(n, r, r);
    double gamma_prev = 0.0, alpha_prev = 0.0;
    int it = 0;
    while (sqrt(rr) > tol * bnorm && it < maxit) {
        block_spmv(nv, rowptr, colidx, vals, u, w);
        double gamma = dotn(n, r, u);
        double delta = dotn(n, w, u);
        double beta = it == 0 ? 0.0 : gamma / gamma_prev;
        double den = it == 0 ? delta : delta - beta * gamma / alpha_prev;
        if (!(den > 0.0)) { out[3] = 1.0; break; }
        double alpha = gamma / den;
        for (int i = 0; i < n; ++i) {
            p[i] = u[i] + beta * p[i];
            s[i] = w[i] + beta * s[i];
            x[i] += alpha * p[i];
            r[i] -= alpha * s[i];
        }
        apply_precond(nv, rowptr, colidx, vals, diag, precond, r, u);
        rr = dotn(n, r, r);
        gamma_prev = gamma;
        alpha_prev = alpha;
        ++it;
    }
    block_spmv(nv, rowptr, colidx, vals, x, w);
    double tr = 0.0;
    for (int i = 0; i < n; ++i) tr += (b[i] - w[i]) * (b[i] - w[i]);
    out[0] = it;
    out[1] = sqrt(rr) / bnorm;
    out[2] = sqrt(tr) / bnorm;
    free(r); free(u); free(w); free(p); free(s);
    return sqrt(rr) <= tol * bnorm ? 0 : 1;
}

/* Jacobi-preconditioned CG (or_pcg2 with precond 0). */
int or_pcg(int nv, const int32_t *rowptr, const int32_t *colidx, const double *vals,
           const double *b, const double *diag, double *x, double tol, int maxit, double *out) {
    return or_pcg2(nv, rowptr, colidx, vals, b, diag, x, tol, maxit, 0, out);
}

/* Run `maxit` CG iterations unconditionally (for timing a bounded sample). */
int or_pcg_fixed(int nv, const int32_t *rowptr, const int32_t *colidx, const double *vals,
                 const double *b, const double *diag, double *x, int iters, double *out) {
    return or_pcg(nv, rowptr, colidx, vals, b, diag, x, 0.0, iters, out);
}

/* Backward-Euler update: v += dv, x += h v (pinned vertices keep x and v = 0). */
void or_update(int nv, const uint8_t *pinned, double h, const double *dv, double *x, double *v) {
    for (int i = 0; i < nv; ++i) {
        if (pinned[i]) { v[3 * i] = v[3 * i + 1] = v[3 * i + 2] = 0.0; continue; }
        for (int a = 0; a < 3; ++a) {
            v[3 * i + a] += dv[3 * i + a];
            x[3 * i + a] += h * v[3 * i + a];
        }
    }
}
