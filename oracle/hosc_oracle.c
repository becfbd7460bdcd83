/*
 * hosc_oracle.c -- plain, slow FP64 CPU oracle of the higher-order super-compact
 * (HOSC) scheme for three-dimensional natural convection of a power-law fluid in a
 * differentially heated cubic cavity (Punia & Ray, arXiv 2411.06563).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no code, header,
 * table or helper with the GPU library; the product never calls it.
 *
 * What it computes, and where the paper defines it:
 *   - strain invariant I2 and power-law viscosity eta            (Sec. 2.1, Eqs. 6-8)
 *   - momentum source terms E* (pressure, eta-gradient, buoyancy) (Sec. 2.1, Eqs. 8-10
 *     in their expanded form, mapped onto the generic PDE as in Sec. 2.2)
 *   - the HOSC time step of the generic transport PDE            (Sec. 2.2, Eqs. 1-5)
 *     written in OPERATOR form: every difference operator is the tensor product of
 *     1D central weights, composed operators are evaluated by that definition, and
 *     the implicit 7-point operator B and the explicit operator A are the bracketed
 *     operators of Eq. 5 multiplied through by L.  The expanded (19,7) weights of
 *     the paper are NOT used here (the GPU path uses them; tests compare).
 *   - linear solves B dchi = b by plain BiCGSTAB (van der Vorst 1992), or by a dense
 *     LU with partial pivoting on tiny grids (brute force)                (Sec. 2.2)
 *   - modified artificial-compressibility pressure correction            (Sec. 2.2)
 *   - Nusselt reductions (Sec. 4.2), entropy generation and Bejan number (Sec. 4.3)
 *
 * Readings of points the paper leaves open or prints garbled (each is also listed
 * in the design notes of the repository):
 *   R1  every term of the momentum source is divided by Pr*eta, so that the generic
 *       PDE keeps its unit coefficient on the Laplacian with L = 1/(Pr eta).
 *   R2  the time-derivative term of L in the compact chi_tt replacement enters with
 *       a minus sign (it comes from d/dt of the generic PDE).
 *   R3  the M18 coefficient is [(dt/2) delta_t^- + sum_d (h_d^2/12)(delta_d^2 - V_d
 *       delta_d)] L  (a "+" is lost in print).
 *   R9  zero normal derivative (theta on the y/z walls, p on all walls) is closed by
 *       f_0 = (4 f_1 - f_2)/3.  theta: for every interior i, first the z walls at
 *       interior j, then the y walls at every k.  p: x faces at interior (j,k), then
 *       y faces at every i and interior k, then z faces at every (i,j).
 *   R10 derivatives of u,v,w,eta,theta at wall nodes are 2nd-order one-sided along
 *       the axis normal to that wall, central along the wall; the wall-normal
 *       derivative of p is zero (the boundary condition).
 *   R11 at the first step level n-1 is taken equal to level n.
 *   R12 eta = max(I2, i2_floor)^((n-1)/2); I2 itself is left raw in E_FF.
 *   R13 buoyancy Ra Pr (theta - theta_ref), theta_ref = 1/2 by default.
 *   R14 lambda defaults to h^2/(3 dt) (chosen by the caller).
 *   R15 pressure iterations within a step (Sec. 2.2): after the momentum solves the
 *       largest |div v^{n+1}| is measured; above div_tol the pressure is corrected
 *       by p <- p - lambda div v and, while fewer than p_iters solves were made,
 *       the sources E* are re-formed from level n with the corrected pressure and
 *       the momentum increments solved again.  p_iters <= 1 is one correction per
 *       step.  Each re-solve starts from level n (never from the trial velocity).
 *   R26 at the first step (R11) the level n-1 sources follow each pressure iterate,
 *       so that their time difference stays zero in every solve of that step.
 *   R27 optional viscosity relaxation for steady-state marching (not in the paper):
 *       the viscosity of level n is r eta(v^n) + (1 - r) times that of level n-1
 *       (level n-1 set, r < 1); r = 1 is the stated scheme.  A steady state is a
 *       fixed point of both.
 *   R16 both sides solve in increment form B dchi = b, b = dt (R - A chi^n).
 *   R17 steady residual per field ||chi^{n+1}-chi^n||_2 / ||chi^{n+1}||_2 over all
 *       nodes.
 *   R18 Bejan number reported both as ratio of integrals and volume mean of ratio.
 *   R19 Nu = -d theta/dx at both walls, 5-point 4th-order one-sided difference.
 *   R20 the undefined fluid-friction weight chi* equals phi* (1e-4).
 *   R24 all four transport solves use level-n coefficients, so they are independent.
 *
 * Storage: every field holds the N^3 nodes of the cube including walls, x fastest:
 * node (i,j,k) at i + N*(j + N*k); h = k = l = 1/(N-1).  x = 0 is the hot wall,
 * y is vertical (buoyancy acts in the v equation).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ID(N, i, j, k) ((size_t)(i) + (size_t)(N) * ((size_t)(j) + (size_t)(N) * (size_t)(k)))

typedef struct {
    int32_t N;          /* nodes per side including walls */
    int32_t maxit;      /* BiCGSTAB iteration cap */
    int32_t dense;      /* nonzero: dense LU instead of BiCGSTAB */
    int32_t p_iters;    /* momentum solves per step at most (pressure iterations, R15); <= 1: one */
    double Ra, Pr, n_pl, dt;
    double theta_hot, theta_cold, theta_ref;
    double lambda, div_tol, i2_floor, phi, solve_tol;
    double eta_relax;   /* weight r of the new viscosity (R27); 1: the stated scheme */
} or_params;

typedef struct {
    double *u, *v, *w, *T, *p;      /* level n */
    double *up, *vp, *wp, *etap;    /* level n-1 */
    double *Eup, *Evp, *Ewp;        /* level n-1 momentum sources */
    int32_t first;                  /* nonzero: level n-1 := level n (reading R11) */
    int32_t pad;
} or_state;

typedef struct {
    double res[4];          /* steady residual of u, v, w, T (reading R17) */
    double maxdiv;          /* max |div v^{n+1}| over interior nodes, before correction */
    double relres[4];       /* final ||b - B dchi|| / ||b|| of each solve */
    int32_t iters[4];       /* solver iterations (0 for dense) */
    int32_t corrected;      /* pressure corrections applied in the step (0 .. p_iters) */
    int32_t status;         /* 0 ok, 1 not converged, 2 non-finite */
} or_info;

/* ------------------------------------------------------------------------- */
/* Difference operators                                                       */
/* ------------------------------------------------------------------------- */

/* 1D central weights at offsets -1, 0, +1 for the identity (order 0), the first
 * difference delta (order 1) and the second difference delta^2 (order 2). */
static void weights1d(int order, double h, double w[3])
{
    if (order == 0) {
        w[0] = 0.0; w[1] = 1.0; w[2] = 0.0;
    } else if (order == 1) {
        w[0] = -0.5 / h; w[1] = 0.0; w[2] = 0.5 / h;
    } else {
        w[0] = 1.0 / (h * h); w[1] = -2.0 / (h * h); w[2] = 1.0 / (h * h);
    }
}

/* delta_x^ox delta_y^oy delta_z^oz f at an interior node: the tensor product of the
 * 1D weights (this is what a composition of central differences means). */
static double Dc(const double *f, int N, double h, int i, int j, int k, int ox, int oy, int oz)
{
    double wx[3], wy[3], wz[3];
    weights1d(ox, h, wx);
    weights1d(oy, h, wy);
    weights1d(oz, h, wz);
    double s = 0.0;
    for (int c = -1; c <= 1; ++c) {
        if (wz[c + 1] == 0.0) continue;
        for (int b = -1; b <= 1; ++b) {
            if (wy[b + 1] == 0.0) continue;
            for (int a = -1; a <= 1; ++a) {
                if (wx[a + 1] == 0.0) continue;
                s += wx[a + 1] * wy[b + 1] * wz[c + 1] * f[ID(N, i + a, j + b, k + c)];
            }
        }
    }
    return s;
}

/* Single-axis helpers. */
static double D1(const double *f, int N, double h, int i, int j, int k, int axis)
{
    return Dc(f, N, h, i, j, k, axis == 0, axis == 1, axis == 2);
}
static double D2(const double *f, int N, double h, int i, int j, int k, int axis)
{
    return Dc(f, N, h, i, j, k, 2 * (axis == 0), 2 * (axis == 1), 2 * (axis == 2));
}

/* d f / d x_axis at any node (reading R10): central inside, 2nd-order one-sided at
 * index 0 and N-1 along that axis. */
static double dwall(const double *f, int N, double h, int i, int j, int k, int axis)
{
    int idx = axis == 0 ? i : axis == 1 ? j : k;
    size_t s = axis == 0 ? 1 : axis == 1 ? (size_t)N : (size_t)N * (size_t)N;
    size_t c = ID(N, i, j, k);
    if (idx == 0) return (-3.0 * f[c] + 4.0 * f[c + s] - f[c + 2 * s]) / (2.0 * h);
    if (idx == N - 1) return (3.0 * f[c] - 4.0 * f[c - s] + f[c - 2 * s]) / (2.0 * h);
    return (f[c + s] - f[c - s]) / (2.0 * h);
}

/* d p / d x_axis: central inside, zero on a wall normal to that axis (boundary
 * condition dp/dn = 0, reading R10). */
static double dpres(const double *p, int N, double h, int i, int j, int k, int axis)
{
    int idx = axis == 0 ? i : axis == 1 ? j : k;
    if (idx == 0 || idx == N - 1) return 0.0;
    size_t s = axis == 0 ? 1 : axis == 1 ? (size_t)N : (size_t)N * (size_t)N;
    size_t c = ID(N, i, j, k);
    return (p[c + s] - p[c - s]) / (2.0 * h);
}

/* ------------------------------------------------------------------------- */
/* Viscosity and momentum sources (Sec. 2.1)                                  */
/* ------------------------------------------------------------------------- */

/* Second invariant of the strain rate (Eq. 8, first use of the label). */
static double strain_I2(const double *u, const double *v, const double *w, int N, double h, int i, int j, int k)
{
    double ux = dwall(u, N, h, i, j, k, 0), uy = dwall(u, N, h, i, j, k, 1), uz = dwall(u, N, h, i, j, k, 2);
    double vx = dwall(v, N, h, i, j, k, 0), vy = dwall(v, N, h, i, j, k, 1), vz = dwall(v, N, h, i, j, k, 2);
    double wx = dwall(w, N, h, i, j, k, 0), wy = dwall(w, N, h, i, j, k, 1), wz = dwall(w, N, h, i, j, k, 2);
    return 2.0 * (ux * ux + vy * vy + wz * wz) + (uz + wx) * (uz + wx) + (uy + vx) * (uy + vx)
           + (vz + wy) * (vz + wy);
}

/* eta = I2^((n-1)/2) (Eq. 7) with the floor of reading R12.  I2 is optional. */
void or_eta_field(const or_params *P, const double *u, const double *v, const double *w, double *eta, double *I2)
{
    int N = P->N;
    double h = 1.0 / (N - 1);
    double ex = 0.5 * (P->n_pl - 1.0);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < N; ++k)
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
                double s = strain_I2(u, v, w, N, h, i, j, k);
                if (I2) I2[ID(N, i, j, k)] = s;
                eta[ID(N, i, j, k)] = pow(fmax(s, P->i2_floor), ex);
            }
}

/* Momentum sources at every node (Eqs. 8-10 divided by Pr*eta, reading R1):
 *   E*_u = L [ -p_x + Pr (2 u_x eta_x + (u_y+v_x) eta_y + (u_z+w_x) eta_z) ]
 *   E*_v = L [ -p_y + Pr ((u_y+v_x) eta_x + 2 v_y eta_y + (v_z+w_y) eta_z) + Ra Pr (T - T_ref) ]
 *   E*_w = L [ -p_z + Pr ((u_z+w_x) eta_x + (v_z+w_y) eta_y + 2 w_z eta_z) ]
 * with L = 1/(Pr eta).  2 eps_ij = u_i,j + u_j,i gives these forms of 2 Pr eps.grad(eta). */
void or_estar_field(const or_params *P, const double *u, const double *v, const double *w, const double *T,
                    const double *p, const double *eta, double *Eu, double *Ev, double *Ew)
{
    int N = P->N;
    double h = 1.0 / (N - 1);
    double Pr = P->Pr;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < N; ++k)
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
                size_t c = ID(N, i, j, k);
                double ux = dwall(u, N, h, i, j, k, 0), uy = dwall(u, N, h, i, j, k, 1), uz = dwall(u, N, h, i, j, k, 2);
                double vx = dwall(v, N, h, i, j, k, 0), vy = dwall(v, N, h, i, j, k, 1), vz = dwall(v, N, h, i, j, k, 2);
                double wx = dwall(w, N, h, i, j, k, 0), wy = dwall(w, N, h, i, j, k, 1), wz = dwall(w, N, h, i, j, k, 2);
                double ex = dwall(eta, N, h, i, j, k, 0), ey = dwall(eta, N, h, i, j, k, 1), ez = dwall(eta, N, h, i, j, k, 2);
                double px = dpres(p, N, h, i, j, k, 0), py = dpres(p, N, h, i, j, k, 1), pz = dpres(p, N, h, i, j, k, 2);
                double L = 1.0 / (Pr * eta[c]);
                Eu[c] = L * (-px + Pr * (2.0 * ux * ex + (uy + vx) * ey + (uz + wx) * ez));
                Ev[c] = L * (-py + Pr * ((uy + vx) * ex + 2.0 * vy * ey + (vz + wy) * ez) + P->Ra * Pr * (T[c] - P->theta_ref));
                Ew[c] = L * (-pz + Pr * ((uz + wx) * ex + (vz + wy) * ey + 2.0 * wz * ez));
            }
}

/* ------------------------------------------------------------------------- */
/* The HOSC operators of the generic transport PDE (Sec. 2.2, Eqs. 1 and 5)   */
/* ------------------------------------------------------------------------- */
/*
 * Generic PDE (Eq. 1, K* = 0 for every equation of the paper):
 *     L chi_t + G* chi_x + H* chi_y + I* chi_z - lap(chi) = E*
 * With V = (G*, H*, I*), the scheme of Eq. 5 multiplied through by L reads
 *     B (chi^{n+1} - chi^n) / dt + A chi^n = R
 * where
 *     B f = (L + M18) f + sum_d [ c_d (delta_d^2 f - V_d delta_d f) + e_d delta_d f ]
 *         c_d = L h_d^2/12 - dt/2,   e_d = (h_d^2/6) delta_d L,
 *         M18 = (dt/2) delta_t^- L + sum_d (h_d^2/12)(delta_d^2 L - V_d delta_d L)
 *     A f = sum_d ( -a_d delta_d^2 f + m_d delta_d f )
 *         - M5 (dxx dyy - H* dxx dy - G* dx dyy - p1 dx dy) f
 *         - M6 (dyy dzz - I* dyy dz - H* dy dzz - q1 dy dz) f
 *         - M7 (dzz dxx - G* dzz dx - I* dz dxx - r1 dz dx) f
 *         a_d = 1 + (h_d^2/12)(V_d^2 - 2 delta_d V_d)           (alpha, beta, gamma)
 *         m_d = P[V_d]                                          (M1, M2, M3)
 *         M5 = (h^2+k^2)/12, M6 = (k^2+l^2)/12, M7 = (l^2+h^2)/12
 *         p1 = -G*H* + 2 (k^2 delta_y G* + h^2 delta_x H*)/(h^2+k^2)   (and q1, r1 alike)
 *     R = P[E*],  P[f] = f + sum_d (h_d^2/12)(delta_d^2 f - V_d delta_d f) + (dt/2) delta_t^- f
 * delta_t^- f = (f^n - f^{n-1})/dt.  All coefficients are at level n.
 */
typedef struct {
    int N;
    double h, dt;
    const double *L, *V[3];         /* level n */
    const double *Lp, *Vp[3];       /* level n-1 */
} coef_t;

/* P[f] at an interior node (bracket operator shared by M1..M3 and R). */
static double P_op(const coef_t *C, const double *f, const double *fp, int i, int j, int k)
{
    int N = C->N;
    double h = C->h;
    size_t c = ID(N, i, j, k);
    double hd2[3] = {h * h, h * h, h * h};      /* h^2, k^2, l^2 */
    double s = f[c];
    for (int d = 0; d < 3; ++d)
        s += hd2[d] / 12.0 * (D2(f, N, h, i, j, k, d) - C->V[d][c] * D1(f, N, h, i, j, k, d));
    s += 0.5 * C->dt * ((f[c] - fp[c]) / C->dt);
    return s;
}

/* (B x) at an interior node. */
static double B_apply_at(const coef_t *C, const double *x, int i, int j, int k)
{
    int N = C->N;
    double h = C->h, dt = C->dt;
    size_t c = ID(N, i, j, k);
    double hd2[3] = {h * h, h * h, h * h};
    double Lc = C->L[c];
    double M18 = 0.5 * dt * ((C->L[c] - C->Lp[c]) / dt);
    for (int d = 0; d < 3; ++d)
        M18 += hd2[d] / 12.0 * (D2(C->L, N, h, i, j, k, d) - C->V[d][c] * D1(C->L, N, h, i, j, k, d));
    double s = (Lc + M18) * x[c];
    for (int d = 0; d < 3; ++d) {
        double cd = Lc * hd2[d] / 12.0 - 0.5 * dt;
        double ed = hd2[d] / 6.0 * D1(C->L, N, h, i, j, k, d);
        s += cd * (D2(x, N, h, i, j, k, d) - C->V[d][c] * D1(x, N, h, i, j, k, d)) + ed * D1(x, N, h, i, j, k, d);
    }
    return s;
}

/* (A chi) at an interior node. */
static double A_apply_at(const coef_t *C, const double *chi, int i, int j, int k)
{
    int N = C->N;
    double h = C->h;
    size_t c = ID(N, i, j, k);
    double hh = h * h, kk = h * h, ll = h * h;     /* h^2, k^2, l^2 of the paper */
    double hd2[3] = {hh, kk, ll};
    double G = C->V[0][c], H = C->V[1][c], I = C->V[2][c];
    double s = 0.0;
    for (int d = 0; d < 3; ++d) {
        double Vd = C->V[d][c];
        double ad = 1.0 + hd2[d] / 12.0 * (Vd * Vd - 2.0 * D1(C->V[d], N, h, i, j, k, d));
        double md = P_op(C, C->V[d], C->Vp[d], i, j, k);
        s += -ad * D2(chi, N, h, i, j, k, d) + md * D1(chi, N, h, i, j, k, d);
    }
    double M5 = (hh + kk) / 12.0, M6 = (kk + ll) / 12.0, M7 = (ll + hh) / 12.0;
    double p1 = -G * H + 2.0 * (kk * D1(C->V[0], N, h, i, j, k, 1) + hh * D1(C->V[1], N, h, i, j, k, 0)) / (hh + kk);
    double q1 = -H * I + 2.0 * (ll * D1(C->V[1], N, h, i, j, k, 2) + kk * D1(C->V[2], N, h, i, j, k, 1)) / (kk + ll);
    double r1 = -I * G + 2.0 * (hh * D1(C->V[2], N, h, i, j, k, 0) + ll * D1(C->V[0], N, h, i, j, k, 2)) / (ll + hh);
    /* Dc(f, ox, oy, oz) = delta_x^ox delta_y^oy delta_z^oz f */
    s -= M5 * (Dc(chi, N, h, i, j, k, 2, 2, 0) - H * Dc(chi, N, h, i, j, k, 2, 1, 0)
               - G * Dc(chi, N, h, i, j, k, 1, 2, 0) - p1 * Dc(chi, N, h, i, j, k, 1, 1, 0));
    s -= M6 * (Dc(chi, N, h, i, j, k, 0, 2, 2) - I * Dc(chi, N, h, i, j, k, 0, 2, 1)
               - H * Dc(chi, N, h, i, j, k, 0, 1, 2) - q1 * Dc(chi, N, h, i, j, k, 0, 1, 1));
    s -= M7 * (Dc(chi, N, h, i, j, k, 2, 0, 2) - G * Dc(chi, N, h, i, j, k, 1, 0, 2)
               - I * Dc(chi, N, h, i, j, k, 2, 0, 1) - r1 * Dc(chi, N, h, i, j, k, 1, 0, 1));
    return s;
}

/* b = dt (R - A chi^n) at every interior node (walls of b are set to 0). */
static void rhs_field(const coef_t *C, const double *E, const double *Ep, const double *chi, double *b)
{
    int N = C->N;
    memset(b, 0, sizeof(double) * (size_t)N * N * N);
#pragma omp parallel for schedule(static)
    for (int k = 1; k < N - 1; ++k)
        for (int j = 1; j < N - 1; ++j)
            for (int i = 1; i < N - 1; ++i) {
                double R = E ? P_op(C, E, Ep, i, j, k) : 0.0;
                b[ID(N, i, j, k)] = C->dt * (R - A_apply_at(C, chi, i, j, k));
            }
}

/* ------------------------------------------------------------------------- */
/* Matrix rows of B and the linear solve                                      */
/* ------------------------------------------------------------------------- */

/* The 7 neighbours in the order centre, x+, x-, y+, y-, z+, z-. */
static const int NB[7][3] = {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};

/* Rows of B at interior nodes, obtained by applying B to unit vectors (the matrix
 * of a linear operator, column by column).  rows[7*r + m] is the weight of
 * neighbour m in interior row r. */
static void B_rows(const coef_t *C, double *rows)
{
    int N = C->N, M = N - 2;
#pragma omp parallel
    {
        double *e = calloc((size_t)N * N * N, sizeof(double));
#pragma omp for schedule(static)
        for (int k = 1; k < N - 1; ++k)
            for (int j = 1; j < N - 1; ++j)
                for (int i = 1; i < N - 1; ++i) {
                    size_t r = (size_t)(i - 1) + (size_t)M * ((size_t)(j - 1) + (size_t)M * (size_t)(k - 1));
                    for (int m = 0; m < 7; ++m) {
                        size_t q = ID(N, i + NB[m][0], j + NB[m][1], k + NB[m][2]);
                        e[q] = 1.0;
                        rows[7 * r + m] = B_apply_at(C, e, i, j, k);
                        e[q] = 0.0;
                    }
                }
        free(e);
    }
}

/* Zero-normal-derivative closure of theta on the y and z walls (reading R9), for
 * every interior i: z walls at interior j first, then y walls at every k. */
static void theta_yz_closure(double *f, int N)
{
    for (int i = 1; i < N - 1; ++i) {
        for (int j = 1; j < N - 1; ++j) {
            f[ID(N, i, j, 0)] = (4.0 * f[ID(N, i, j, 1)] - f[ID(N, i, j, 2)]) / 3.0;
            f[ID(N, i, j, N - 1)] = (4.0 * f[ID(N, i, j, N - 2)] - f[ID(N, i, j, N - 3)]) / 3.0;
        }
        for (int k = 0; k < N; ++k) {
            f[ID(N, i, 0, k)] = (4.0 * f[ID(N, i, 1, k)] - f[ID(N, i, 2, k)]) / 3.0;
            f[ID(N, i, N - 1, k)] = (4.0 * f[ID(N, i, N - 2, k)] - f[ID(N, i, N - 3, k)]) / 3.0;
        }
    }
}

/* Zero-normal-derivative closure of p on all walls (reading R9): x faces at
 * interior (j,k), then y faces at every i and interior k, then z faces everywhere. */
static void pressure_closure(double *p, int N)
{
    for (int k = 1; k < N - 1; ++k)
        for (int j = 1; j < N - 1; ++j) {
            p[ID(N, 0, j, k)] = (4.0 * p[ID(N, 1, j, k)] - p[ID(N, 2, j, k)]) / 3.0;
            p[ID(N, N - 1, j, k)] = (4.0 * p[ID(N, N - 2, j, k)] - p[ID(N, N - 3, j, k)]) / 3.0;
        }
    for (int k = 1; k < N - 1; ++k)
        for (int i = 0; i < N; ++i) {
            p[ID(N, i, 0, k)] = (4.0 * p[ID(N, i, 1, k)] - p[ID(N, i, 2, k)]) / 3.0;
            p[ID(N, i, N - 1, k)] = (4.0 * p[ID(N, i, N - 2, k)] - p[ID(N, i, N - 3, k)]) / 3.0;
        }
    for (int j = 0; j < N; ++j)
        for (int i = 0; i < N; ++i) {
            p[ID(N, i, j, 0)] = (4.0 * p[ID(N, i, j, 1)] - p[ID(N, i, j, 2)]) / 3.0;
            p[ID(N, i, j, N - 1)] = (4.0 * p[ID(N, i, j, N - 2)] - p[ID(N, i, j, N - 3)]) / 3.0;
        }
}

typedef struct {
    int N;
    const double *rows;     /* 7 weights per interior row */
    int neumann_yz;         /* 1: unknown is theta increment (y/z walls by closure) */
    double *full;           /* N^3 scratch */
} sysop_t;

/* y = B x for an interior vector x: embed x with zero x-walls (Dirichlet), close
 * the y/z walls when the unknown is a temperature increment, apply the rows. */
static void sys_apply(const sysop_t *S, const double *x, double *y)
{
    int N = S->N, M = N - 2;
    double *f = S->full;
    memset(f, 0, sizeof(double) * (size_t)N * N * N);
    for (int k = 1; k < N - 1; ++k)
        for (int j = 1; j < N - 1; ++j)
            for (int i = 1; i < N - 1; ++i)
                f[ID(N, i, j, k)] = x[(size_t)(i - 1) + (size_t)M * ((size_t)(j - 1) + (size_t)M * (size_t)(k - 1))];
    if (S->neumann_yz) theta_yz_closure(f, N);
#pragma omp parallel for schedule(static)
    for (int k = 1; k < N - 1; ++k)
        for (int j = 1; j < N - 1; ++j)
            for (int i = 1; i < N - 1; ++i) {
                size_t r = (size_t)(i - 1) + (size_t)M * ((size_t)(j - 1) + (size_t)M * (size_t)(k - 1));
                double s = 0.0;
                for (int m = 0; m < 7; ++m)
                    s += S->rows[7 * r + m] * f[ID(N, i + NB[m][0], j + NB[m][1], k + NB[m][2])];
                y[r] = s;
            }
}

static double dot(const double *a, const double *b, size_t n)
{
    double s = 0.0;
    for (size_t q = 0; q < n; ++q) s += a[q] * b[q];
    return s;
}

/* Plain BiCGSTAB (van der Vorst 1992) from x = 0, restarted when a scalar of the
 * recurrence breaks down; stops when ||b - B x|| <= tol ||b|| (true residual). */
static int bicgstab(const sysop_t *S, const double *b, double *x, double tol, int maxit, double *relres, int *iters)
{
    size_t n = (size_t)(S->N - 2) * (S->N - 2) * (S->N - 2);
    double *r = malloc(n * sizeof(double)), *rh = malloc(n * sizeof(double));
    double *p = malloc(n * sizeof(double)), *v = malloc(n * sizeof(double));
    double *s = malloc(n * sizeof(double)), *t = malloc(n * sizeof(double));
    double bn = sqrt(dot(b, b, n));
    int status = 1, it = 0;
    memset(x, 0, n * sizeof(double));
    if (bn == 0.0) {
        *relres = 0.0; *iters = 0; status = 0;
        goto done;
    }
    while (it < maxit) {
        /* (re)start from the current iterate */
        sys_apply(S, x, t);
        for (size_t q = 0; q < n; ++q) { r[q] = b[q] - t[q]; rh[q] = r[q]; p[q] = 0.0; v[q] = 0.0; }
        double rn = sqrt(dot(r, r, n));
        if (rn <= tol * bn) { status = 0; *relres = rn / bn; break; }
        double rho = 1.0, alpha = 1.0, omega = 1.0;
        int restart = 0;
        while (it < maxit && !restart) {
            ++it;
            double rho1 = dot(rh, r, n);
            if (fabs(rho1) < 1e-300 || !isfinite(rho1)) { restart = 1; break; }
            double beta = (rho1 / rho) * (alpha / omega);
            for (size_t q = 0; q < n; ++q) p[q] = r[q] + beta * (p[q] - omega * v[q]);
            sys_apply(S, p, v);
            double rv = dot(rh, v, n);
            if (fabs(rv) < 1e-300 || !isfinite(rv)) { restart = 1; break; }
            alpha = rho1 / rv;
            for (size_t q = 0; q < n; ++q) s[q] = r[q] - alpha * v[q];
            double sn = sqrt(dot(s, s, n));
            if (sn <= tol * bn) {
                for (size_t q = 0; q < n; ++q) x[q] += alpha * p[q];
                restart = 1;   /* confirm with the true residual */
                break;
            }
            sys_apply(S, s, t);
            double tt = dot(t, t, n);
            if (tt == 0.0 || !isfinite(tt)) { for (size_t q = 0; q < n; ++q) x[q] += alpha * p[q]; restart = 1; break; }
            omega = dot(t, s, n) / tt;
            for (size_t q = 0; q < n; ++q) { x[q] += alpha * p[q] + omega * s[q]; r[q] = s[q] - omega * t[q]; }
            rho = rho1;
            rn = sqrt(dot(r, r, n));
            if (!isfinite(rn)) { status = 2; *relres = NAN; *iters = it; goto done; }
            if (rn <= tol * bn) { restart = 1; break; }   /* confirm with the true residual */
            if (omega == 0.0) { restart = 1; break; }
        }
    }
    if (status != 0) {
        sys_apply(S, x, t);
        for (size_t q = 0; q < n; ++q) r[q] = b[q] - t[q];
        double rn = sqrt(dot(r, r, n));
        *relres = rn / bn;
        status = isfinite(rn) ? (rn <= tol * bn ? 0 : 1) : 2;
    }
    *iters = it;
done:
    free(r); free(rh); free(p); free(v); free(s); free(t);
    return status;
}

/* Brute force: dense matrix of the operator (columns = images of unit vectors) and
 * LU with partial pivoting. */
static int dense_solve(const sysop_t *S, const double *b, double *x, double *relres)
{
    size_t n = (size_t)(S->N - 2) * (S->N - 2) * (S->N - 2);
    double *A = malloc(n * n * sizeof(double));
    double *e = calloc(n, sizeof(double)), *col = malloc(n * sizeof(double));
    for (size_t c = 0; c < n; ++c) {
        e[c] = 1.0;
        sys_apply(S, e, col);
        e[c] = 0.0;
        for (size_t r = 0; r < n; ++r) A[r * n + c] = col[r];
    }
    double *y = malloc(n * sizeof(double));
    memcpy(y, b, n * sizeof(double));
    int status = 0;
    for (size_t c = 0; c < n; ++c) {
        size_t piv = c;
        for (size_t r = c + 1; r < n; ++r)
            if (fabs(A[r * n + c]) > fabs(A[piv * n + c])) piv = r;
        if (A[piv * n + c] == 0.0) { status = 2; break; }
        if (piv != c) {
            for (size_t q = 0; q < n; ++q) { double tq = A[c * n + q]; A[c * n + q] = A[piv * n + q]; A[piv * n + q] = tq; }
            double ty = y[c]; y[c] = y[piv]; y[piv] = ty;
        }
        for (size_t r = c + 1; r < n; ++r) {
            double f = A[r * n + c] / A[c * n + c];
            if (f == 0.0) continue;
            for (size_t q = c; q < n; ++q) A[r * n + q] -= f * A[c * n + q];
            y[r] -= f * y[c];
        }
    }
    if (status == 0)
        for (size_t c = n; c-- > 0;) {
            double s = y[c];
            for (size_t q = c + 1; q < n; ++q) s -= A[c * n + q] * x[q];
            x[c] = s / A[c * n + c];
        }
    /* report the true relative residual */
    sys_apply(S, x, col);
    double rn = 0.0, bn = 0.0;
    for (size_t r = 0; r < n; ++r) { rn += (b[r] - col[r]) * (b[r] - col[r]); bn += b[r] * b[r]; }
    *relres = bn > 0.0 ? sqrt(rn / bn) : 0.0;
    free(A); free(e); free(col); free(y);
    return status;
}

/* Solve B dchi = b for the interior increment; the result is written into the
 * interior of the N^3 field d (walls untouched). */
static int solve_increment(const or_params *P, const double *rows, int neumann_yz, const double *bfull, double *d,
                           double *relres, int *iters)
{
    int N = P->N, M = N - 2;
    size_t n = (size_t)M * M * M;
    double *b = malloc(n * sizeof(double)), *x = malloc(n * sizeof(double));
    for (int k = 1; k < N - 1; ++k)
        for (int j = 1; j < N - 1; ++j)
            for (int i = 1; i < N - 1; ++i)
                b[(size_t)(i - 1) + (size_t)M * ((size_t)(j - 1) + (size_t)M * (size_t)(k - 1))] = bfull[ID(N, i, j, k)];
    sysop_t S = {N, rows, neumann_yz, malloc(sizeof(double) * (size_t)N * N * N)};
    int status;
    *iters = 0;
    if (P->dense)
        status = dense_solve(&S, b, x, relres);
    else
        status = bicgstab(&S, b, x, P->solve_tol, P->maxit, relres, iters);
    for (int k = 1; k < N - 1; ++k)
        for (int j = 1; j < N - 1; ++j)
            for (int i = 1; i < N - 1; ++i)
                d[ID(N, i, j, k)] = x[(size_t)(i - 1) + (size_t)M * ((size_t)(j - 1) + (size_t)M * (size_t)(k - 1))];
    free(S.full); free(b); free(x);
    return status;
}

/* ------------------------------------------------------------------------- */
/* Boundary conditions (Sec. 2.1)                                             */
/* ------------------------------------------------------------------------- */

/* Impose the boundary conditions on a state: no-slip velocity on every wall,
 * theta = theta_hot at x = 0 and theta_cold at x = 1, zero normal derivative of
 * theta on the y/z walls and of p on every wall (reading R9). */
void or_apply_bc(const or_params *P, double *u, double *v, double *w, double *T, double *p)
{
    int N = P->N;
    for (int k = 0; k < N; ++k)
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
                int wall = i == 0 || j == 0 || k == 0 || i == N - 1 || j == N - 1 || k == N - 1;
                if (!wall) continue;
                size_t c = ID(N, i, j, k);
                if (u) u[c] = 0.0;
                if (v) v[c] = 0.0;
                if (w) w[c] = 0.0;
                if (T && i == 0) T[c] = P->theta_hot;
                if (T && i == N - 1) T[c] = P->theta_cold;
            }
    if (T) theta_yz_closure(T, N);
    if (p) pressure_closure(p, N);
}

/* ------------------------------------------------------------------------- */
/* One time step                                                              */
/* ------------------------------------------------------------------------- */

static double field_res(const double *a, const double *b, size_t n)
{
    double num = 0.0, den = 0.0;
    for (size_t q = 0; q < n; ++q) { num += (b[q] - a[q]) * (b[q] - a[q]); den += b[q] * b[q]; }
    if (den > 0.0) return sqrt(num) / sqrt(den);
    return num == 0.0 ? 0.0 : INFINITY;
}

/* Coefficient fields of the energy equation (L = 1, V = (u, v, w), E* = 0) and of
 * the momentum equations (L = 1/(Pr eta), V = (u, v, w) L), Sec. 2.2. */
typedef struct {
    double *Lm, *Gm, *Hm, *Im, *Lmp, *Gmp, *Hmp, *Imp;   /* momentum, levels n and n-1 */
    double *one;
} coef_store_t;

/* Outputs of the assembly stage, for the parity tests:
 *   b[4] (u, v, w, T increments' right-hand sides) and the coefficient fields. */
static void build_coefs(const or_params *P, const or_state *S, const double *eta, coef_store_t *cs, coef_t *Cm,
                        coef_t *Ct)
{
    int N = P->N;
    size_t n3 = (size_t)N * N * N;
    double h = 1.0 / (N - 1);
    for (size_t q = 0; q < n3; ++q) {
        cs->Lm[q] = 1.0 / (P->Pr * eta[q]);
        cs->Gm[q] = S->u[q] * cs->Lm[q];
        cs->Hm[q] = S->v[q] * cs->Lm[q];
        cs->Im[q] = S->w[q] * cs->Lm[q];
        cs->Lmp[q] = 1.0 / (P->Pr * S->etap[q]);
        cs->Gmp[q] = S->up[q] * cs->Lmp[q];
        cs->Hmp[q] = S->vp[q] * cs->Lmp[q];
        cs->Imp[q] = S->wp[q] * cs->Lmp[q];
        cs->one[q] = 1.0;
    }
    Cm->N = N; Cm->h = h; Cm->dt = P->dt;
    Cm->L = cs->Lm; Cm->V[0] = cs->Gm; Cm->V[1] = cs->Hm; Cm->V[2] = cs->Im;
    Cm->Lp = cs->Lmp; Cm->Vp[0] = cs->Gmp; Cm->Vp[1] = cs->Hmp; Cm->Vp[2] = cs->Imp;
    Ct->N = N; Ct->h = h; Ct->dt = P->dt;
    Ct->L = cs->one; Ct->V[0] = S->u; Ct->V[1] = S->v; Ct->V[2] = S->w;
    Ct->Lp = cs->one; Ct->Vp[0] = S->up; Ct->Vp[1] = S->vp; Ct->Vp[2] = S->wp;
}

static void coef_alloc(coef_store_t *cs, size_t n3)
{
    double **f[9] = {&cs->Lm, &cs->Gm, &cs->Hm, &cs->Im, &cs->Lmp, &cs->Gmp, &cs->Hmp, &cs->Imp, &cs->one};
    for (int q = 0; q < 9; ++q) *f[q] = malloc(n3 * sizeof(double));
}
static void coef_free(coef_store_t *cs)
{
    free(cs->Lm); free(cs->Gm); free(cs->Hm); free(cs->Im);
    free(cs->Lmp); free(cs->Gmp); free(cs->Hmp); free(cs->Imp); free(cs->one);
}

/* Viscosity of level n: eta(v^n), relaxed towards level n-1 when asked (R27). */
static void level_eta(const or_params *P, const or_state *S, double *eta)
{
    size_t n3 = (size_t)P->N * P->N * P->N;
    or_eta_field(P, S->u, S->v, S->w, eta, NULL);
    if (!S->first && P->eta_relax < 1.0)
        for (size_t c = 0; c < n3; ++c) eta[c] = P->eta_relax * eta[c] + (1.0 - P->eta_relax) * S->etap[c];
}

/* Level-n viscosity and sources, and level n-1 set equal on the first step. */
static void stage_sources(const or_params *P, or_state *S, double *eta, double *Eu, double *Ev, double *Ew)
{
    size_t n3 = (size_t)P->N * P->N * P->N;
    level_eta(P, S, eta);
    or_estar_field(P, S->u, S->v, S->w, S->T, S->p, eta, Eu, Ev, Ew);
    if (S->first) {
        memcpy(S->up, S->u, n3 * sizeof(double));
        memcpy(S->vp, S->v, n3 * sizeof(double));
        memcpy(S->wp, S->w, n3 * sizeof(double));
        memcpy(S->etap, eta, n3 * sizeof(double));
        memcpy(S->Eup, Eu, n3 * sizeof(double));
        memcpy(S->Evp, Ev, n3 * sizeof(double));
        memcpy(S->Ewp, Ew, n3 * sizeof(double));
        S->first = 0;
    }
}

/* Assembly only (for parity tests): right-hand sides b of the u, v, w and T
 * increment systems (b4 = 4 N^3 arrays, walls 0), and optionally eta, E*.
 * The state is not advanced; level n-1 is taken equal to level n when first is set
 * (the state's level n-1 arrays are then overwritten with level n). */
int or_assemble(const or_params *P, or_state *S, double *b4, double *eta_out, double *E3_out)
{
    int N = P->N;
    size_t n3 = (size_t)N * N * N;
    double *eta = malloc(n3 * sizeof(double));
    double *Eu = malloc(n3 * sizeof(double)), *Ev = malloc(n3 * sizeof(double)), *Ew = malloc(n3 * sizeof(double));
    stage_sources(P, S, eta, Eu, Ev, Ew);
    coef_store_t cs;
    coef_alloc(&cs, n3);
    coef_t Cm, Ct;
    build_coefs(P, S, eta, &cs, &Cm, &Ct);
    rhs_field(&Cm, Eu, S->Eup, S->u, b4);
    rhs_field(&Cm, Ev, S->Evp, S->v, b4 + n3);
    rhs_field(&Cm, Ew, S->Ewp, S->w, b4 + 2 * n3);
    rhs_field(&Ct, NULL, NULL, S->T, b4 + 3 * n3);
    if (eta_out) memcpy(eta_out, eta, n3 * sizeof(double));
    if (E3_out) {
        memcpy(E3_out, Eu, n3 * sizeof(double));
        memcpy(E3_out + n3, Ev, n3 * sizeof(double));
        memcpy(E3_out + 2 * n3, Ew, n3 * sizeof(double));
    }
    coef_free(&cs);
    free(eta); free(Eu); free(Ev); free(Ew);
    return 0;
}

/* y = B x at interior nodes (walls of y set to 0) for the momentum operator
 * (eq = 0) or the energy operator (eq = 1) of the given state; x is used as given
 * (no closure), so this is the raw 7-point operator.  Level n-1 must be set. */
int or_apply_B(const or_params *P, const or_state *S, int eq, const double *x, double *y)
{
    int N = P->N;
    size_t n3 = (size_t)N * N * N;
    double *eta = malloc(n3 * sizeof(double));
    level_eta(P, S, eta);
    coef_store_t cs;
    coef_alloc(&cs, n3);
    coef_t Cm, Ct;
    build_coefs(P, S, eta, &cs, &Cm, &Ct);
    const coef_t *C = eq == 0 ? &Cm : &Ct;
    memset(y, 0, n3 * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int k = 1; k < N - 1; ++k)
        for (int j = 1; j < N - 1; ++j)
            for (int i = 1; i < N - 1; ++i) y[ID(N, i, j, k)] = B_apply_at(C, x, i, j, k);
    coef_free(&cs);
    free(eta);
    return 0;
}

/* One HOSC time step (Sec. 2.2): viscosity and sources from level n, the four
 * increment solves, the pressure iterations of the modified artificial-
 * compressibility method (momentum re-solved after each correction, R15), the
 * update with boundary conditions and the steady residual; level n becomes level
 * n-1. */
int or_step(const or_params *P, or_state *S, or_info *info)
{
    int N = P->N, M = N - 2;
    size_t n3 = (size_t)N * N * N;
    double h = 1.0 / (N - 1);
    const int first = S->first;
    double *eta = malloc(n3 * sizeof(double));
    double *E[3] = {malloc(n3 * sizeof(double)), malloc(n3 * sizeof(double)), malloc(n3 * sizeof(double))};
    stage_sources(P, S, eta, E[0], E[1], E[2]);

    coef_store_t cs;
    coef_alloc(&cs, n3);
    coef_t Cm, Ct;
    build_coefs(P, S, eta, &cs, &Cm, &Ct);

    double *chi[4] = {S->u, S->v, S->w, S->T};
    double *Ep[3] = {S->Eup, S->Evp, S->Ewp};
    double *b = malloc(4 * n3 * sizeof(double));
    for (int q = 0; q < 3; ++q) rhs_field(&Cm, E[q], Ep[q], chi[q], b + q * n3);
    rhs_field(&Ct, NULL, NULL, S->T, b + 3 * n3);

    double *rows_m = malloc(7 * (size_t)M * M * M * sizeof(double));
    double *rows_t = malloc(7 * (size_t)M * M * M * sizeof(double));
    B_rows(&Cm, rows_m);
    B_rows(&Ct, rows_t);

    /* energy: its coefficients and sources do not involve the pressure (R24) */
    double *d = calloc(4 * n3, sizeof(double));
    int status = solve_increment(P, rows_t, 1, b + 3 * n3, d + 3 * n3, &info->relres[3], &info->iters[3]);

    /* momentum with pressure iterations: trial velocity level n + increment, its
     * divergence, and a correction of p followed by a re-solve while allowed */
    const int K = P->p_iters > 1 ? P->p_iters : 1;
    double *trial[3] = {malloc(n3 * sizeof(double)), malloc(n3 * sizeof(double)), malloc(n3 * sizeof(double))};
    double *div = calloc(n3, sizeof(double));
    double maxdiv = 0.0;
    info->corrected = 0;
    for (int q = 0; q < 3; ++q) info->iters[q] = 0;
    for (int it = 0;; ++it) {
        for (int q = 0; q < 3; ++q) {
            int iters = 0;
            int st = solve_increment(P, rows_m, 0, b + q * n3, d + q * n3, &info->relres[q], &iters);
            info->iters[q] += iters;
            if (st > status) status = st;
            memcpy(trial[q], chi[q], n3 * sizeof(double));
            for (int k = 1; k < N - 1; ++k)
                for (int j = 1; j < N - 1; ++j)
                    for (int i = 1; i < N - 1; ++i) trial[q][ID(N, i, j, k)] += d[q * n3 + ID(N, i, j, k)];
        }
        maxdiv = 0.0;
        for (int k = 1; k < N - 1; ++k)
            for (int j = 1; j < N - 1; ++j)
                for (int i = 1; i < N - 1; ++i) {
                    double D = D1(trial[0], N, h, i, j, k, 0) + D1(trial[1], N, h, i, j, k, 1)
                               + D1(trial[2], N, h, i, j, k, 2);
                    div[ID(N, i, j, k)] = D;
                    if (fabs(D) > maxdiv || isnan(D)) maxdiv = isnan(D) ? NAN : fabs(D);
                }
        if (!(maxdiv > P->div_tol)) break;      /* accurate enough (or non-finite) */
        /* p <- p - lambda div v at interior nodes, walls by the zero-gradient closure */
        for (int k = 1; k < N - 1; ++k)
            for (int j = 1; j < N - 1; ++j)
                for (int i = 1; i < N - 1; ++i) S->p[ID(N, i, j, k)] -= P->lambda * div[ID(N, i, j, k)];
        pressure_closure(S->p, N);
        info->corrected += 1;
        if (it + 1 >= K) break;
        /* sources of level n with the corrected pressure; eta is unchanged */
        or_estar_field(P, S->u, S->v, S->w, S->T, S->p, eta, E[0], E[1], E[2]);
        if (first)
            for (int q = 0; q < 3; ++q) memcpy(Ep[q], E[q], n3 * sizeof(double));
        for (int q = 0; q < 3; ++q) rhs_field(&Cm, E[q], Ep[q], chi[q], b + q * n3);
    }
    info->maxdiv = maxdiv;

    /* level n becomes level n-1 */
    memcpy(S->up, S->u, n3 * sizeof(double));
    memcpy(S->vp, S->v, n3 * sizeof(double));
    memcpy(S->wp, S->w, n3 * sizeof(double));
    memcpy(S->etap, eta, n3 * sizeof(double));
    memcpy(S->Eup, E[0], n3 * sizeof(double));
    memcpy(S->Evp, E[1], n3 * sizeof(double));
    memcpy(S->Ewp, E[2], n3 * sizeof(double));

    /* update chi^{n+1} = chi^n + dchi: the accepted trial velocity, theta at interior
     * nodes and then its walls */
    double *old = malloc(4 * n3 * sizeof(double));
    for (int q = 0; q < 4; ++q) memcpy(old + q * n3, chi[q], n3 * sizeof(double));
    for (int q = 0; q < 3; ++q) memcpy(chi[q], trial[q], n3 * sizeof(double));
    for (int k = 1; k < N - 1; ++k)
        for (int j = 1; j < N - 1; ++j)
            for (int i = 1; i < N - 1; ++i) S->T[ID(N, i, j, k)] += d[3 * n3 + ID(N, i, j, k)];
    theta_yz_closure(S->T, N);
    for (int q = 0; q < 4; ++q) info->res[q] = field_res(old + q * n3, chi[q], n3);

    for (int q = 0; q < 4; ++q)
        if (!isfinite(info->res[q])) status = 2;
    if (!isfinite(maxdiv)) status = 2;
    info->status = status;

    free(trial[0]); free(trial[1]); free(trial[2]);
    free(div); free(old); free(d); free(rows_m); free(rows_t); free(b);
    coef_free(&cs);
    free(eta); free(E[0]); free(E[1]); free(E[2]);
    return status;
}

/* ------------------------------------------------------------------------- */
/* Generic transport step (test hook for manufactured solutions)              */
/* ------------------------------------------------------------------------- */

/* One HOSC step of the generic PDE (Eq. 1) with caller-supplied coefficient fields
 * at levels n and n-1 (all N^3 nodes), Dirichlet data: the walls of chi_new must
 * hold the level n+1 boundary values on entry; its interior is overwritten.
 * G, H, I are the convective coefficients G*, H*, I*.  E may be NULL (zero). */
int or_transport_step(const or_params *P, const double *L, const double *G, const double *H, const double *I,
                      const double *E, const double *Lp, const double *Gp, const double *Hp, const double *Ip,
                      const double *Ep, const double *chi, double *chi_new, double *relres, int *iters)
{
    int N = P->N, M = N - 2;
    size_t n3 = (size_t)N * N * N;
    coef_t C = {N, 1.0 / (N - 1), P->dt, L, {G, H, I}, Lp, {Gp, Hp, Ip}};
    double *b = malloc(n3 * sizeof(double));
    rhs_field(&C, E, Ep, chi, b);
    /* wall increments are known: move B(dchi_wall) to the right-hand side */
    double *dw = calloc(n3, sizeof(double));
    for (int k = 0; k < N; ++k)
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
                int wall = i == 0 || j == 0 || k == 0 || i == N - 1 || j == N - 1 || k == N - 1;
                if (wall) dw[ID(N, i, j, k)] = chi_new[ID(N, i, j, k)] - chi[ID(N, i, j, k)];
            }
    for (int k = 1; k < N - 1; ++k)
        for (int j = 1; j < N - 1; ++j)
            for (int i = 1; i < N - 1; ++i) b[ID(N, i, j, k)] -= B_apply_at(&C, dw, i, j, k);
    double *rows = malloc(7 * (size_t)M * M * M * sizeof(double));
    B_rows(&C, rows);
    double *d = calloc(n3, sizeof(double));
    int st = solve_increment(P, rows, 0, b, d, relres, iters);
    for (int k = 1; k < N - 1; ++k)
        for (int j = 1; j < N - 1; ++j)
            for (int i = 1; i < N - 1; ++i) chi_new[ID(N, i, j, k)] = chi[ID(N, i, j, k)] + d[ID(N, i, j, k)];
    free(b); free(dw); free(rows); free(d);
    return st;
}

/* ------------------------------------------------------------------------- */
/* Nusselt, entropy generation and Bejan number (Secs. 4.2, 4.3)              */
/* ------------------------------------------------------------------------- */

/* Composite Simpson weights on N equally spaced nodes of [0, 1]; when N-1 is odd
 * the last three intervals use Simpson's 3/8 rule. */
static void simpson_weights(int N, double *wq)
{
    double h = 1.0 / (N - 1);
    int nint = N - 1;
    for (int q = 0; q < N; ++q) wq[q] = 0.0;
    int n13 = (nint % 2 == 0) ? nint : nint - 3;     /* intervals covered by the 1/3 rule */
    for (int q = 0; q < n13; q += 2) {
        wq[q] += h / 3.0; wq[q + 1] += 4.0 * h / 3.0; wq[q + 2] += h / 3.0;
    }
    if (n13 != nint) {
        int q = n13;
        wq[q] += 3.0 * h / 8.0; wq[q + 1] += 9.0 * h / 8.0; wq[q + 2] += 9.0 * h / 8.0; wq[q + 3] += 3.0 * h / 8.0;
    }
}

/* Outputs (any pointer may be NULL except scal):
 *   nu_hot, nu_cold [N*N, index j + N*k]: local Nu = -dtheta/dx on x = 0 and x = 1
 *   nuavg_hot, nuavg_cold [N]: Nu_avg(z) = int_0^1 Nu dy
 *   scal[10] = { Nu_mean_hot, Nu_mean_cold, Nu_max_hot (max_z Nu_avg), Nu_max_cold,
 *                E_total, int E_HT, int E_FF, Be_global, Be_mean, max Nu_local hot }
 *   e_local, be_local [N^3]: local entropy generation and local Bejan number. */
int or_diagnostics(const or_params *P, const double *u, const double *v, const double *w, const double *T,
                   double *nu_hot, double *nu_cold, double *nuavg_hot, double *nuavg_cold, double *scal,
                   double *e_local, double *be_local)
{
    int N = P->N;
    double h = 1.0 / (N - 1);
    double *wq = malloc(N * sizeof(double));
    simpson_weights(N, wq);
    double *nh = malloc((size_t)N * N * sizeof(double)), *nc = malloc((size_t)N * N * sizeof(double));
    double numax_local = -INFINITY;
    for (int k = 0; k < N; ++k)
        for (int j = 0; j < N; ++j) {
            /* 5-point 4th-order one-sided first derivative (reading R19) */
            double dh = (-25.0 * T[ID(N, 0, j, k)] + 48.0 * T[ID(N, 1, j, k)] - 36.0 * T[ID(N, 2, j, k)]
                         + 16.0 * T[ID(N, 3, j, k)] - 3.0 * T[ID(N, 4, j, k)]) / (12.0 * h);
            double dc = (25.0 * T[ID(N, N - 1, j, k)] - 48.0 * T[ID(N, N - 2, j, k)] + 36.0 * T[ID(N, N - 3, j, k)]
                         - 16.0 * T[ID(N, N - 4, j, k)] + 3.0 * T[ID(N, N - 5, j, k)]) / (12.0 * h);
            nh[j + (size_t)N * k] = -dh;
            nc[j + (size_t)N * k] = -dc;
            if (-dh > numax_local) numax_local = -dh;
        }
    double mean_h = 0.0, mean_c = 0.0, max_h = -INFINITY, max_c = -INFINITY;
    for (int k = 0; k < N; ++k) {
        double ah = 0.0, ac = 0.0;
        for (int j = 0; j < N; ++j) { ah += wq[j] * nh[j + (size_t)N * k]; ac += wq[j] * nc[j + (size_t)N * k]; }
        if (nuavg_hot) nuavg_hot[k] = ah;
        if (nuavg_cold) nuavg_cold[k] = ac;
        if (ah > max_h) max_h = ah;
        if (ac > max_c) max_c = ac;
        mean_h += wq[k] * ah;
        mean_c += wq[k] * ac;
    }
    if (nu_hot) memcpy(nu_hot, nh, (size_t)N * N * sizeof(double));
    if (nu_cold) memcpy(nu_cold, nc, (size_t)N * N * sizeof(double));

    /* entropy generation (Eqs. of Sec. 4.3) with eta from the current velocity */
    size_t n3 = (size_t)N * N * N;
    double *eta = malloc(n3 * sizeof(double)), *I2 = malloc(n3 * sizeof(double));
    or_eta_field(P, u, v, w, eta, I2);
    double s_ht = 0.0, s_ff = 0.0, s_be = 0.0;
    for (int k = 0; k < N; ++k)
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i) {
                size_t c = ID(N, i, j, k);
                double tx = dwall(T, N, h, i, j, k, 0), ty = dwall(T, N, h, i, j, k, 1), tz = dwall(T, N, h, i, j, k, 2);
                double eht = tx * tx + ty * ty + tz * tz;
                double eff = P->phi * eta[c] * I2[c];
                double el = eht + eff;
                double be = el > 0.0 ? eht / el : 1.0;
                double wv = wq[i] * wq[j] * wq[k];
                s_ht += wv * eht;
                s_ff += wv * eff;
                s_be += wv * be;
                if (e_local) e_local[c] = el;
                if (be_local) be_local[c] = be;
            }
    scal[0] = mean_h; scal[1] = mean_c; scal[2] = max_h; scal[3] = max_c;
    scal[4] = s_ht + s_ff; scal[5] = s_ht; scal[6] = s_ff;
    scal[7] = (s_ht + s_ff) > 0.0 ? s_ht / (s_ht + s_ff) : 1.0;
    scal[8] = s_be;
    scal[9] = numax_local;
    free(eta); free(I2); free(wq); free(nh); free(nc);
    return 0;
}

/* Number of OpenMP threads the oracle's node loops use (1 without OpenMP). */
#ifdef _OPENMP
#include <omp.h>
int or_num_threads(void) { return omp_get_max_threads(); }
#else
int or_num_threads(void) { return 1; }
#endif
