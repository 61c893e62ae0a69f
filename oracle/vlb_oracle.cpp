/*
 * vlb_oracle.cpp -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, double-precision CPU implementation of one coupled time step of the
 * viscoelastic lattice Boltzmann method of Yu, Chen, Wang, Yuan and Shu, "An improved
 * lattice Boltzmann method with a novel conservative boundary scheme for viscoelastic
 * fluid flows" (arXiv:2508.16997).  It exists to check the HIP library: only the tests,
 * the package smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the library.
 *
 * Every step follows the paper's equations in the paper's order, with the Hermite
 * tensor sums written out over all index combinations (no D2Q9 shortcuts), one pass
 * over the grid per stage, state stored as absolute populations:
 *
 *   1. macroscopic density and velocity with the half-force shift    (Sec. 3.1)
 *   2. conformation components and polymer stress (Kramers relation with the
 *      model function F(A): Oldroyd-B, Giesekus, PTT, FENE-P)           (Sec. 2.2-2.3)
 *   3. velocity gradient and d(rho u^3) by finite differences           (reading A6/A7)
 *   4. constitutive source Phi_ab                                         (Sec. 3.2)
 *   5. hydrodynamic TRT regularized collision with G_i, F_i, T_i         (Sec. 3.1)
 *   6. three convection-diffusion TRT regularized collisions with
 *      the auxiliary source, the source term and its time derivative   (Sec. 3.2)
 *   7. streaming; half-way / linearly interpolated bounce-back for f, or the
 *      unified interpolation with the rest-population mass restore      (reading A30);
 *      non-equilibrium extrapolation at the inlet and outlet ghosts    (readings A13, A21)
 *      or, for wet-node walls, non-equilibrium bounce-back of f at the wall nodes
 *      themselves (Sec. 4.2-4.3, reading A29)
 *   8. conservative non-equilibrium bounce-back for every g lattice     (Sec. 3.3)
 *   9. history of S and u for the backward time difference             (Sec. 3.2)
 *
 * plus the momentum-exchange force on solids (Sec. 4.3).
 *
 * Readings of points the paper leaves open are listed in the repository's design
 * notes under the same labels (A5 ... A25) and are marked where they are used.
 *
 * The solver is templated on the scalar type so that a forward-mode dual number can
 * carry exact derivatives with respect to lambda, eta_p and the body-force field.
 * Geometry (node classes, links, wall fractions q) is always plain double.
 *
 * Build: g++ -O2 -std=c++17 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math).
 */
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ----------------------------------------------------------------------------------
// Dual number for forward-mode derivatives (value v, tangent d).
// ----------------------------------------------------------------------------------
struct Dual {
    double v, d;
    Dual() : v(0), d(0) {}
    Dual(double a) : v(a), d(0) {}
    Dual(double a, double b) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
    return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v));
}
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
inline double val(double a) { return a; }
inline double val(const Dual& a) { return a.v; }
inline double tan_(double) { return 0.0; }
inline double tan_(const Dual& a) { return a.d; }

// ----------------------------------------------------------------------------------
// D2Q9 lattice (Sec. 3.1): velocities e_i from the paper's cos/sin formula,
// weights 4/9, 1/9 (i = 1..4), 1/36 (i = 5..8), c_s^2 = 1/3.
// ----------------------------------------------------------------------------------
const int Q = 9;
int EX[Q], EY[Q], OPP[Q];
const double W[Q] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                     1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
const double CS2 = 1.0 / 3.0;

struct LatticeInit {
    LatticeInit() {
        const double pi = std::acos(-1.0);
        EX[0] = 0; EY[0] = 0;
        for (int i = 1; i <= 4; ++i) {
            EX[i] = (int)std::lround(std::cos(pi * (i - 1) / 2.0));
            EY[i] = (int)std::lround(std::sin(pi * (i - 1) / 2.0));
        }
        for (int i = 5; i <= 8; ++i) {
            EX[i] = (int)std::lround(std::sqrt(2.0) * std::cos(pi * (i - 4.5) / 2.0));
            EY[i] = (int)std::lround(std::sqrt(2.0) * std::sin(pi * (i - 4.5) / 2.0));
        }
        for (int i = 0; i < Q; ++i)
            for (int j = 0; j < Q; ++j)
                if (EX[j] == -EX[i] && EY[j] == -EY[i]) OPP[i] = j;
    }
} lattice_init_instance;

inline double ec(int i, int a) { return a == 0 ? (double)EX[i] : (double)EY[i]; }
inline double kd(int a, int b) { return a == b ? 1.0 : 0.0; }

// Hermite polynomials of orders 1..3 (order 0 is 1), Sec. 3.1.
inline double H1(int i, int a) { return ec(i, a); }
inline double H2(int i, int a, int b) { return ec(i, a) * ec(i, b) - CS2 * kd(a, b); }
inline double H3(int i, int a, int b, int c) {
    return ec(i, a) * ec(i, b) * ec(i, c) -
           CS2 * (ec(i, a) * kd(b, c) + ec(i, b) * kd(a, c) + ec(i, c) * kd(a, b));
}

// Hydrodynamic equilibrium, third-order Hermite expansion (Sec. 3.1).
template <class R>
R feq(int i, R rho, R ux, R uy) {
    const R u[2] = {ux, uy};
    R s = R(1.0);
    for (int a = 0; a < 2; ++a) s += R(H1(i, a) / CS2) * u[a];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) s += R(H2(i, a, b) / (2.0 * CS2 * CS2)) * u[a] * u[b];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 2; ++c)
                s += R(H3(i, a, b, c) / (6.0 * CS2 * CS2 * CS2)) * u[a] * u[b] * u[c];
    return R(W[i]) * rho * s;
}

// Convection-diffusion equilibrium, second-order Hermite expansion (Sec. 3.2).
template <class R>
R geq(int i, R phi, R ux, R uy) {
    const R u[2] = {ux, uy};
    R s = R(1.0);
    for (int a = 0; a < 2; ++a) s += R(H1(i, a) / CS2) * u[a];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) s += R(H2(i, a, b) / (2.0 * CS2 * CS2)) * u[a] * u[b];
    return R(W[i]) * phi * s;
}

template <class R>
struct Relax {
    R tau_s1, tau_s2, tau_p1, tau_p2, lam, eta_p;
};

// Hydrodynamic TRT regularized collision (Sec. 3.1): off-equilibrium moments of
// orders 0..3, tau_s1 on orders 0..2 and tau_s2 on order 3, plus the Galilean
// correction G_i, the body-force term F_i and the viscoelastic source T_i (dt = 1).
// A_0 and A_a are computed literally from f - f^eq (reading A5).
template <class R>
void collide_hydro(const R f[Q], R rho, R ux, R uy, R Fx, R Fy, const R tau_ab[2][2],
                   R Dx, R Dy, const Relax<R>& p, R out[Q]) {
    R fe[Q];
    for (int i = 0; i < Q; ++i) fe[i] = feq(i, rho, ux, uy);
    R A0 = R(0.0), A1[2] = {R(0.0), R(0.0)};
    R A2[2][2] = {{R(0.0), R(0.0)}, {R(0.0), R(0.0)}};
    R A3[2][2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 2; ++c) A3[a][b][c] = R(0.0);
    for (int i = 0; i < Q; ++i) {
        const R d = f[i] - fe[i];
        A0 += d;
        for (int a = 0; a < 2; ++a) A1[a] += R(H1(i, a)) * d;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) A2[a][b] += R(H2(i, a, b)) * d;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int c = 0; c < 2; ++c) A3[a][b][c] += R(H3(i, a, b, c)) * d;
    }
    // d_gamma Phi_abg: only (x,x) <- d_x(rho ux^3) and (y,y) <- d_y(rho uy^3).
    const R dPhi[2][2] = {{Dx, R(0.0)}, {R(0.0), Dy}};
    const R F[2] = {Fx, Fy};
    const R one = R(1.0);
    const R c1 = one - one / p.tau_s1;
    const R c2 = one - one / p.tau_s2;
    const R h1 = one - one / (R(2.0) * p.tau_s1);
    for (int i = 0; i < Q; ++i) {
        R reg1 = A0;
        for (int a = 0; a < 2; ++a) reg1 += R(H1(i, a) / CS2) * A1[a];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) reg1 += R(H2(i, a, b) / (2.0 * CS2 * CS2)) * A2[a][b];
        R reg2 = R(0.0);
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                for (int c = 0; c < 2; ++c)
                    reg2 += R(H3(i, a, b, c) / (6.0 * CS2 * CS2 * CS2)) * A3[a][b][c];
        R sumG = R(0.0), sumT = R(0.0), sumF = R(0.0);
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                sumG += R(H2(i, a, b) / (6.0 * CS2 * CS2 * CS2)) * dPhi[a][b];
                sumT += R(H2(i, a, b) / (2.0 * CS2 * CS2)) * tau_ab[a][b];
            }
        for (int a = 0; a < 2; ++a) sumF += R(H1(i, a) / CS2) * F[a];
        const R Gi = -R(W[i]) * h1 * sumG;
        const R Ti = -R(W[i]) * sumT / p.tau_s1;
        const R Fi = h1 * R(W[i]) * sumF;
        out[i] = fe[i] + R(W[i]) * c1 * reg1 + R(W[i]) * c2 * reg2 + Gi + Fi + Ti;
    }
}

// Convection-diffusion TRT regularized collision for one scalar phi (Sec. 3.2):
// tau_p1 on orders 0..1, tau_p2 on order 2, auxiliary term G~_i (incompressible form,
// reading A8), source term F~_i and its backward time difference (dt = 1).
template <class R>
void collide_cde(const R g[Q], R phi, R rho, R ux, R uy, R Fx, R Fy, R S, R Sp, R uxp,
                 R uyp, const Relax<R>& p, R out[Q]) {
    R ge[Q];
    for (int i = 0; i < Q; ++i) ge[i] = geq(i, phi, ux, uy);
    R B0 = R(0.0), B1[2] = {R(0.0), R(0.0)};
    R B2[2][2] = {{R(0.0), R(0.0)}, {R(0.0), R(0.0)}};
    for (int i = 0; i < Q; ++i) {
        const R d = g[i] - ge[i];
        B0 += d;
        for (int a = 0; a < 2; ++a) B1[a] += R(H1(i, a)) * d;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) B2[a][b] += R(H2(i, a, b)) * d;
    }
    const R one = R(1.0);
    const R c1 = one - one / p.tau_p1;
    const R c2 = one - one / p.tau_p2;
    const R h2 = one - one / (R(2.0) * p.tau_p1);
    const R F[2] = {Fx, Fy};
    const R u[2] = {ux, uy};
    const R up[2] = {uxp, uyp};
    for (int i = 0; i < Q; ++i) {
        R reg1 = B0;
        for (int a = 0; a < 2; ++a) reg1 += R(H1(i, a) / CS2) * B1[a];
        R reg2 = R(0.0);
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) reg2 += R(H2(i, a, b) / (2.0 * CS2 * CS2)) * B2[a][b];
        R eF = R(0.0), eu = R(0.0), eup = R(0.0);
        for (int a = 0; a < 2; ++a) {
            eF += R(ec(i, a) / CS2) * F[a];
            eu += R(ec(i, a) / CS2) * u[a];
            eup += R(ec(i, a) / CS2) * up[a];
        }
        const R Gt = R(W[i]) * h2 * eF * phi / rho;
        const R Ft_now = R(W[i]) * S + h2 * R(W[i]) * eu * S;
        const R Ft_prev = R(W[i]) * Sp + h2 * R(W[i]) * eup * Sp;
        const R dtFt = Ft_now - Ft_prev;
        out[i] = ge[i] + R(W[i]) * c1 * reg1 + R(W[i]) * c2 * reg2 + Gt + Ft_now +
                 R(0.5) * dtFt;
    }
}

// Constitutive models enter only through the model function F(A) (Sec. 2.2: the
// conformation equation relaxes with -(1/lambda) F and the Kramers relation gives the
// polymer stress (eta_p / lambda) F).  The paper runs the Oldroyd-B closure
// F = A - I.  The other closures it names are written here in the conformation form:
// a relaxation function F_r (in the transport equation) and a stress function F_s (in
// the Kramers relation), with the 2-D trace tr A (equal to 2 at rest):
//   Giesekus (alpha):    F_r = (A - I) + alpha (A - I)^2,           F_s = A - I
//   linear PTT (eps):    F_r = [1 + eps (tr A - 2)] (A - I),        F_s = A - I
//   exponential PTT:     F_r = exp[eps (tr A - 2)] (A - I),         F_s = A - I
//   FENE-P (L^2):        F_r = F_s = f A - I,  f = (L^2 - 2) / (L^2 - tr A)
enum { MODEL_OLDROYD_B = 0, MODEL_GIESEKUS = 1, MODEL_LPTT = 2, MODEL_EPTT = 3, MODEL_FENE_P = 4 };

inline double exp_(double a) { return std::exp(a); }
inline Dual exp_(Dual a) {
    const double e = std::exp(a.v);
    return Dual(e, e * a.d);
}

template <class R>
void model_functions(const R A[2][2], int model, double mp, R Fr[2][2], R Fs[2][2]) {
    R B[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) B[a][b] = A[a][b] - R(kd(a, b));
    const R trA = A[0][0] + A[1][1];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            Fs[a][b] = B[a][b];
            Fr[a][b] = B[a][b];
        }
    if (model == MODEL_GIESEKUS) {
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                R bb = R(0.0);
                for (int g = 0; g < 2; ++g) bb += B[a][g] * B[g][b];
                Fr[a][b] = B[a][b] + R(mp) * bb;
            }
    } else if (model == MODEL_LPTT || model == MODEL_EPTT) {
        const R x = R(mp) * (trA - R(2.0));
        const R Y = model == MODEL_LPTT ? R(1.0) + x : exp_(x);
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) Fr[a][b] = Y * B[a][b];
    } else if (model == MODEL_FENE_P) {
        const R f = R(mp - 2.0) / (R(mp) - trA);
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                Fr[a][b] = f * A[a][b] - R(kd(a, b));
                Fs[a][b] = Fr[a][b];
            }
    }
}

// Constitutive source Phi_ab (Sec. 3.2), with L[g][b] = d_g u_b:
// -F_r(A)/lambda + A_ag L_gb + A_gb L_ga + A_ab L_gg.
template <class R>
void constitutive_source(const R A[2][2], const R L[2][2], R lam, int model, double mp,
                         R S[2][2]) {
    R Fr[2][2], Fs[2][2];
    model_functions(A, model, mp, Fr, Fs);
    const R trL = L[0][0] + L[1][1];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            R s = -Fr[a][b] / lam;
            for (int g = 0; g < 2; ++g) s += A[a][g] * L[g][b] + A[g][b] * L[g][a];
            s += A[a][b] * trL;
            S[a][b] = s;
        }
}

// Finite-difference derivative along one axis (reading A6): central difference
// between the two neighbours, or the quadratic through the no-slip wall value 0 at
// fraction q when a neighbour is solid.
template <class R>
R fd_axis(bool lo_solid, double qlo, R plo, R p0, bool hi_solid, double qhi, R phi) {
    if (!lo_solid && !hi_solid) return (phi - plo) * R(0.5);
    if (lo_solid && !hi_solid)
        return R(qlo / (1.0 + qlo)) * phi + R((1.0 - qlo) / qlo) * p0;
    if (!lo_solid && hi_solid)
        return -(R(qhi / (1.0 + qhi)) * plo + R((1.0 - qhi) / qhi) * p0);
    return p0 * R((qhi - qlo) / (qlo * qhi));
}

// MODE_WET (y only): the first and last rows are wall nodes (wet-node walls, u = 0 on
// them, channel height ny - 1; reading A29).
enum { MODE_PERIODIC = 0, MODE_WALL = 1, MODE_OPEN = 2, MODE_WET = 3 };
enum { SRC_FLUID = 0, SRC_SOLID = 1, SRC_INLET = 2, SRC_OUTLET = 3 };
// FLAG_NO_GTILDE drops the auxiliary term G~_i of the convection-diffusion collision: a
// planted mistake for the sensitivity checks of the tests, never the method.
// FLAG_CNEBB_UB_ZERO and FLAG_CNEBB_PAIR_NEQ are the alternative readings of two points
// the boundary scheme of Sec. 3.3 leaves open, kept only to measure how much the result
// depends on them: the velocity in the CNEBB equilibrium taken as the wall's (zero)
// instead of the boundary node's (reading A11), and an unknown population whose opposite
// is unknown too rebuilt with the non-equilibrium part of the population that left in
// its own direction instead of the equilibrium alone (reading A12).
// FLAG_CURVED_YLW selects the paper's curved-wall scheme for the hydrodynamic lattice on
// the cylinder (Sec. 4.3, "YLW", reading A30) instead of linear interpolated bounce-back:
// the unified interpolation of Yu, Mei, Luo and Shyy (2003) on links with q != 1/2, and
// the rest population restoring the local mass (known populations plus those that left
// toward the wall), the conservation strategy CNEBB shares with it (Sec. 3.3).
// FLAG_OPEN_NEBB selects the paper's hydrodynamic open ends of the cylinder (Sec. 4.3,
// reading A31): the first and last columns are wet boundary nodes whose populations from
// beyond the inlet / outlet are rebuilt by non-equilibrium bounce-back (Zou-He) for the
// inlet velocity (u_in(y), 0) and for the reference density 1 with u_y = 0 at the outlet;
// the conformation lattices keep the non-equilibrium extrapolation ghosts.
enum { FLAG_NO_SOURCE = 1, FLAG_NO_GTILDE = 2, FLAG_CNEBB_UB_ZERO = 4, FLAG_CNEBB_PAIR_NEQ = 8,
       FLAG_CURVED_YLW = 16, FLAG_OPEN_NEBB = 32 };

struct Src {
    int kind;
    int node;  // source node (fluid, outlet copy) or -1
    int ys;    // source row (inlet/outlet ghosts)
    double q;  // wall fraction along the link (solid)
};

struct Geometry {
    int nx = 0, ny = 0, xmode = 0, ymode = 0;
    std::vector<uint8_t> solid;   // 1 = solid (mask or inside a circle)
    std::vector<int> circle_of;   // circle containing the node, or -1
    std::vector<double> circ;     // xc, yc, R per circle

    static int wrap(int v, int n) { return ((v % n) + n) % n; }

    void build(int nx_, int ny_, int xm, int ym, const uint8_t* mask, const double* circles,
               int ncirc) {
        nx = nx_; ny = ny_; xmode = xm; ymode = ym;
        solid.assign((size_t)nx * ny, 0);
        circle_of.assign((size_t)nx * ny, -1);
        circ.assign(circles, circles + 3 * ncirc);
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const size_t n = (size_t)y * nx + x;
                if (mask && mask[n]) solid[n] = 1;
                for (int c = 0; c < ncirc; ++c) {
                    const double dx = (double)x - circ[3 * c];
                    const double dy = (double)y - circ[3 * c + 1];
                    const double r = circ[3 * c + 2];
                    if (dx * dx + dy * dy <= r * r) {
                        solid[n] = 1;
                        if (circle_of[n] < 0) circle_of[n] = c;
                    }
                }
            }
    }

    // Wall fraction of the link from fluid node (x, y) toward solid node x - e_i: the
    // smallest root t of |x + t d - c|^2 = R^2 with d = -e_i (reading A23); 1/2 for
    // solids that are not inside a circle.
    double link_q(int x, int y, int i, int s) const {
        const int c = circle_of[s];
        if (c < 0) return 0.5;
        const double dx = -(double)EX[i], dy = -(double)EY[i];
        const double px = (double)x - circ[3 * c], py = (double)y - circ[3 * c + 1];
        const double r = circ[3 * c + 2];
        const double a = dx * dx + dy * dy;
        const double b = 2.0 * (px * dx + py * dy);
        const double cc = px * px + py * py - r * r;
        const double disc = b * b - 4.0 * a * cc;
        return (-b - std::sqrt(disc)) / (2.0 * a);
    }

    // Where the population moving in direction i into (x, y) comes from: x - e_i.
    Src source(int x, int y, int i) const {
        int xs = x - EX[i], ys = y - EY[i];
        const bool xout = xs < 0 || xs >= nx, yout = ys < 0 || ys >= ny;
        if ((yout && (ymode == MODE_WALL || ymode == MODE_WET)) || (xout && xmode == MODE_WALL))
            return Src{SRC_SOLID, -1, -1, 0.5};
        if (yout) ys = wrap(ys, ny);
        if (xout) {
            if (xmode == MODE_PERIODIC) xs = wrap(xs, nx);
            else if (xs < 0) return Src{SRC_INLET, -1, ys, 0.0};
            else return Src{SRC_OUTLET, ys * nx + (nx - 1), ys, 0.0};
        }
        const int s = ys * nx + xs;
        if (solid[s]) return Src{SRC_SOLID, s, ys, link_q(x, y, i, s)};
        return Src{SRC_FLUID, s, ys, 0.0};
    }

    // Wall node of a wet-node wall: first or last row.
    bool wet_row(int y) const { return ymode == MODE_WET && (y == 0 || y == ny - 1); }

    bool is_boundary(int x, int y) const {
        for (int i = 1; i < Q; ++i)
            if (source(x, y, i).kind == SRC_SOLID) return true;
        return false;
    }
};

template <class R>
struct Sim {
    Geometry geo;
    int nx = 0, ny = 0;
    size_t N = 0;
    Relax<R> p{};
    int flags = 0;
    int model = MODEL_OLDROYD_B;  // constitutive closure and its parameter
    double mpar = 0.0;
    std::vector<R> Fx, Fy;
    std::vector<R> uin, ain[3];
    std::vector<R> f[Q], fp[Q], g[3][Q], gp[3][Q];
    std::vector<R> Sprev[3], uxp, uyp;
    std::vector<R> rho, ux, uy, A[3];  // macroscopic fields at the current time
    bool first = true;
    long long step = 0;

    void alloc() {
        N = (size_t)nx * ny;
        for (int i = 0; i < Q; ++i) {
            f[i].assign(N, R(0.0)); fp[i].assign(N, R(0.0));
            for (int k = 0; k < 3; ++k) { g[k][i].assign(N, R(0.0)); gp[k][i].assign(N, R(0.0)); }
        }
        for (int k = 0; k < 3; ++k) { Sprev[k].assign(N, R(0.0)); A[k].assign(N, R(0.0)); }
        uxp.assign(N, R(0.0)); uyp.assign(N, R(0.0));
        rho.assign(N, R(0.0)); ux.assign(N, R(0.0)); uy.assign(N, R(0.0));
        Fx.assign(N, R(0.0)); Fy.assign(N, R(0.0));
        uin.assign(ny, R(0.0));
        for (int k = 0; k < 3; ++k) ain[k].assign(ny, R(0.0));
    }

    bool fluid(size_t n) const { return geo.solid[n] == 0; }

    // Stage 1-2: rho, u with the half-force shift (Sec. 3.1) and A from the g lattices.
    void macros() {
#pragma omp parallel for schedule(static)
        for (long long nn = 0; nn < (long long)N; ++nn) {
            const size_t n = (size_t)nn;
            if (!fluid(n)) continue;
            R r = R(0.0), jx = R(0.0), jy = R(0.0);
            for (int i = 0; i < Q; ++i) {
                r += f[i][n];
                jx += R((double)EX[i]) * f[i][n];
                jy += R((double)EY[i]) * f[i][n];
            }
            rho[n] = r;
            ux[n] = (jx + R(0.5) * Fx[n]) / r;
            uy[n] = (jy + R(0.5) * Fy[n]) / r;
            if (geo.wet_row((int)(n / nx))) {  // wall node: the wall velocity (reading A29)
                ux[n] = R(0.0);
                uy[n] = R(0.0);
            }
            for (int k = 0; k < 3; ++k) {
                R s = R(0.0);
                for (int i = 0; i < Q; ++i) s += g[k][i][n];
                A[k][n] = s;
            }
        }
    }

    // Value of a field at a neighbour for the finite differences (reading A6): fluid
    // node, inlet ghost (prescribed profile, rho = 1), outlet ghost (copy of the last
    // column, zero gradient).
    template <class Fn>
    R nb_value(const Src& s, Fn field_at, R inlet_value) const {
        if (s.kind == SRC_INLET) return inlet_value;
        return field_at(s.node);
    }

    void step_once() {
        macros();
        std::vector<R> Snew[3];
        for (int k = 0; k < 3; ++k) Snew[k].assign(N, R(0.0));
        // Stages 3-6, node by node.
#pragma omp parallel for schedule(static)
        for (long long nn = 0; nn < (long long)N; ++nn) {
            const size_t n = (size_t)nn;
            if (!fluid(n)) continue;
            const int x = (int)(n % nx), y = (int)(n / nx);
            // Neighbours along the axes are the sources of directions 1 (x-1), 3 (x+1),
            // 2 (y-1) and 4 (y+1).
            const Src sxl = geo.source(x, y, 1), sxh = geo.source(x, y, 3);
            const Src syl = geo.source(x, y, 2), syh = geo.source(x, y, 4);
            auto ux_at = [&](int m) { return ux[m]; };
            auto uy_at = [&](int m) { return uy[m]; };
            auto px_at = [&](int m) { return rho[m] * ux[m] * ux[m] * ux[m]; };
            auto py_at = [&](int m) { return rho[m] * uy[m] * uy[m] * uy[m]; };
            auto D = [&](const Src& lo, const Src& hi, auto fn, R p0, R inl_lo, R inl_hi) {
                const bool ls = lo.kind == SRC_SOLID, hs = hi.kind == SRC_SOLID;
                const R vlo = ls ? R(0.0) : nb_value(lo, fn, inl_lo);
                const R vhi = hs ? R(0.0) : nb_value(hi, fn, inl_hi);
                return fd_axis(ls, lo.q, vlo, p0, hs, hi.q, vhi);
            };
            const R uinl = sxl.kind == SRC_INLET ? uin[sxl.ys] : R(0.0);
            R L[2][2];
            L[0][0] = D(sxl, sxh, ux_at, ux[n], uinl, R(0.0));
            L[0][1] = D(sxl, sxh, uy_at, uy[n], R(0.0), R(0.0));
            L[1][0] = D(syl, syh, ux_at, ux[n], R(0.0), R(0.0));
            L[1][1] = D(syl, syh, uy_at, uy[n], R(0.0), R(0.0));
            const R Dx = D(sxl, sxh, px_at, rho[n] * ux[n] * ux[n] * ux[n],
                           uinl * uinl * uinl, R(0.0));
            R Dy = D(syl, syh, py_at, rho[n] * uy[n] * uy[n] * uy[n], R(0.0), R(0.0));
            if (geo.wet_row(y)) {
                // Wall node of a wet-node wall: wall-normal derivatives by the one-sided
                // second-order difference through the node and the next two rows into the
                // fluid (reading A29).
                const int s1 = y == 0 ? 1 : -1;
                const size_t n1 = (size_t)(y + s1) * nx + x, n2 = (size_t)(y + 2 * s1) * nx + x;
                auto one_sided = [&](auto fn, R p0) {
                    return R((double)s1) * (R(-1.5) * p0 + R(2.0) * fn(n1) - R(0.5) * fn(n2));
                };
                L[1][0] = one_sided(ux_at, ux[n]);
                L[1][1] = one_sided(uy_at, uy[n]);
                Dy = one_sided(py_at, rho[n] * uy[n] * uy[n] * uy[n]);
            }

            // Conformation tensor and polymer stress tau = (eta_p / lambda) F_s(A).
            const R Am[2][2] = {{A[0][n], A[1][n]}, {A[1][n], A[2][n]}};
            R Fr[2][2], Fs[2][2], tau_ab[2][2];
            model_functions(Am, model, mpar, Fr, Fs);
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) tau_ab[a][b] = p.eta_p / p.lam * Fs[a][b];
            R Sm[2][2];
            constitutive_source(Am, L, p.lam, model, mpar, Sm);
            R S[3] = {Sm[0][0], Sm[0][1], Sm[1][1]};
            if (flags & FLAG_NO_SOURCE) S[0] = S[1] = S[2] = R(0.0);
            // First step: F~(t - 1) := F~(t) (reading A9).
            R Sp[3], uxprev, uyprev;
            for (int k = 0; k < 3; ++k) Sp[k] = first ? S[k] : Sprev[k][n];
            uxprev = first ? ux[n] : uxp[n];
            uyprev = first ? uy[n] : uyp[n];

            R fl[Q], out[Q];
            for (int i = 0; i < Q; ++i) fl[i] = f[i][n];
            collide_hydro(fl, rho[n], ux[n], uy[n], Fx[n], Fy[n], tau_ab, Dx, Dy, p, out);
            for (int i = 0; i < Q; ++i) fp[i][n] = out[i];
            for (int k = 0; k < 3; ++k) {
                R gl[Q];
                for (int i = 0; i < Q; ++i) gl[i] = g[k][i][n];
                // (the body force enters the convection-diffusion collision only through
                // G~_i)
                const bool gt = !(flags & FLAG_NO_GTILDE);
                collide_cde(gl, A[k][n], rho[n], ux[n], uy[n], gt ? Fx[n] : R(0.0),
                            gt ? Fy[n] : R(0.0), S[k], Sp[k], uxprev, uyprev, p, out);
                for (int i = 0; i < Q; ++i) gp[k][i][n] = out[i];
                Snew[k][n] = S[k];
            }
        }
        // Stage 7: streaming with the hydrodynamic wall fill and the open ghosts.
#pragma omp parallel for schedule(static)
        for (long long nn = 0; nn < (long long)N; ++nn) {
            const size_t n = (size_t)nn;
            if (!fluid(n)) continue;
            const int x = (int)(n % nx), y = (int)(n / nx);
            for (int i = 0; i < Q; ++i) {
                const Src s = geo.source(x, y, i);
                const int o = OPP[i];
                if (s.kind == SRC_FLUID) {
                    f[i][n] = fp[i][s.node];
                    for (int k = 0; k < 3; ++k) g[k][i][n] = gp[k][i][s.node];
                } else if (s.kind == SRC_INLET || s.kind == SRC_OUTLET) {
                    // Open ends (reading A21): non-equilibrium extrapolation from the node
                    // x0 next to the ghost (first or last column, same row): its
                    // post-collision populations minus their own equilibrium, plus the
                    // equilibrium of the boundary state -- inlet: rho(x0) and the inlet
                    // profile (u_in, A_in); outlet: rho = 1 and u(x0) for the hydrodynamic
                    // lattice, a plain copy of x0 for the conformation lattices.
                    const bool in = s.kind == SRC_INLET;
                    const size_t m = in ? (size_t)s.ys * nx : (size_t)s.node;
                    if (!fluid(m)) {
                        f[i][n] = feq(i, R(1.0), in ? uin[s.ys] : R(0.0), R(0.0));
                        for (int k = 0; k < 3; ++k)
                            g[k][i][n] = geq(i, in ? ain[k][s.ys] : R(k == 1 ? 0.0 : 1.0), in ? uin[s.ys] : R(0.0), R(0.0));
                        continue;
                    }
                    R r = R(0.0), jx = R(0.0), jy = R(0.0);
                    for (int j = 0; j < Q; ++j) {
                        r += fp[j][m];
                        jx += R((double)EX[j]) * fp[j][m];
                        jy += R((double)EY[j]) * fp[j][m];
                    }
                    const R vx = jx / r, vy = jy / r;
                    const R fneq = fp[i][m] - feq(i, r, vx, vy);
                    f[i][n] = in ? feq(i, r, uin[s.ys], R(0.0)) + fneq : feq(i, R(1.0), vx, vy) + fneq;
                    for (int k = 0; k < 3; ++k) {
                        if (!in) {
                            g[k][i][n] = gp[k][i][m];
                            continue;
                        }
                        R ph = R(0.0);
                        for (int j = 0; j < Q; ++j) ph += gp[k][j][m];
                        g[k][i][n] = geq(i, ain[k][s.ys], uin[s.ys], R(0.0)) + gp[k][i][m] -
                                     geq(i, ph, vx, vy);
                    }
                } else {
                    // Hydrodynamic wall: half-way bounce-back for q = 1/2 (reading A13),
                    // linear interpolated bounce-back otherwise (reading A21), or the
                    // unified scheme (reading A30).
                    const double q = s.q;
                    if (q == 0.5) {
                        f[i][n] = fp[o][n];
                    } else if (flags & FLAG_CURVED_YLW) {
                        // The population that left x toward the wall in direction o meets
                        // it at distance q.  Linear interpolation along the link between
                        // where the direction-o populations sit after streaming -- x (from
                        // the far node x + e_i) and the solid node (from x) -- gives the
                        // value at the wall point; bounced there, it is interpolated back
                        // to x with the direction-i population streamed from x to x + e_i
                        // (one spacing on the other side):
                        //   f_o(wall) = (1 - q) fp_o(x + e_i) + q fp_o(x)
                        //   f_i(x) = [f_o(wall) + q fp_i(x)] / (1 + q).
                        // Without a fluid far node: half-way bounce-back.
                        const Src far = geo.source(x, y, o);  // x - e_o = x + e_i
                        if (far.kind == SRC_FLUID)
                            f[i][n] = (R(1.0 - q) * fp[o][far.node] + R(q) * fp[o][n] +
                                       R(q) * fp[i][n]) / R(1.0 + q);
                        else
                            f[i][n] = fp[o][n];
                    } else if (q < 0.5) {
                        const Src far = geo.source(x, y, o);  // x - e_o = x + e_i
                        if (far.kind == SRC_FLUID)
                            f[i][n] = R(2.0 * q) * fp[o][n] + R(1.0 - 2.0 * q) * fp[o][far.node];
                        else
                            f[i][n] = fp[o][n];
                    } else {
                        f[i][n] = R(1.0 / (2.0 * q)) * fp[o][n] +
                                  R((2.0 * q - 1.0) / (2.0 * q)) * fp[i][n];
                    }
                    // Conformation lattices: the populations that left toward the wall,
                    // used for phi at the boundary node; replaced by CNEBB below.
                    for (int k = 0; k < 3; ++k) g[k][i][n] = gp[k][o][n];
                }
            }
        }
        // Stage 7a (reading A30): the rest population of a wall-adjacent node takes the
        // mass the interpolation did not return -- the node's density after streaming is
        // its known populations plus the post-collision populations that left toward
        // the wall.
        if (flags & FLAG_CURVED_YLW) {
#pragma omp parallel for schedule(static)
            for (long long nn = 0; nn < (long long)N; ++nn) {
                const size_t n = (size_t)nn;
                if (!fluid(n)) continue;
                const int x = (int)(n % nx), y = (int)(n / nx);
                for (int i = 1; i < Q; ++i)
                    if (geo.source(x, y, i).kind == SRC_SOLID) f[0][n] += fp[OPP[i]][n] - f[i][n];
            }
        }
        // Stage 7c (reading A31): wet-node open ends.  At the inlet column the three
        // populations arriving from x < 0 (e_x = +1) are unknown.  The density follows
        // from the known ones and the prescribed velocity: with K the sum of the rest,
        // tangential and twice the outgoing populations, the streamed momentum
        // j_x = rho u_in - F_x/2 (half-force shift) gives rho = (K - F_x/2) / (1 - u_in).
        // The normal unknown keeps the non-equilibrium part of its opposite; the two
        // diagonal ones then follow from the x and y momentum balances
        // (j_y = -F_y/2, no transverse velocity).  At the outlet column the same with the
        // roles of +x and -x exchanged and the density prescribed (1): j_x = K - 1.
        // At a corner with a wet-node wall the wall rule (stage 7b) follows and has the
        // last word.
        if (geo.xmode == MODE_OPEN && (flags & FLAG_OPEN_NEBB)) {
#pragma omp parallel for schedule(static)
            for (long long yy = 0; yy < (long long)ny; ++yy) {
                for (int side = 0; side < 2; ++side) {
                    const int x = side == 0 ? 0 : nx - 1;
                    const size_t n = (size_t)yy * nx + (size_t)x;
                    if (!fluid(n)) continue;
                    const int sx = side == 0 ? 1 : -1;  // unknown directions have e_x = sx
                    R K = R(0.0);
                    for (int i = 0; i < Q; ++i) {
                        if (EX[i] == 0) K += f[i][n];
                        else if (EX[i] == -sx) K += R(2.0) * f[i][n];
                    }
                    R r, jx;
                    if (side == 0) {
                        r = (K - R(0.5) * Fx[n]) / (R(1.0) - uin[yy]);
                        jx = r * uin[yy] - R(0.5) * Fx[n];
                    } else {
                        r = R(1.0);
                        jx = K - r;
                    }
                    const R jy = R(-0.5) * Fy[n];
                    // normal: f_n - f_opp(n) = 2 w_n 3 e_n.j (the equilibrium difference)
                    const int in = sx > 0 ? 1 : 3;
                    f[in][n] = f[OPP[in]][n] + R(2.0 * W[in] * 3.0 * sx) * jx;
                    // diagonals (a: e_y = +1, b: e_y = -1): solve
                    //   sx (f_a + f_b) = jx - [sum_{e_x != 0, known} e_x f] - sx f_n
                    //   f_a - f_b = jy - [sum_{e_y != 0, not a, b} e_y f]
                    int ia = -1, ib = -1;
                    for (int i = 0; i < Q; ++i)
                        if (EX[i] == sx && EY[i] == 1) ia = i;
                        else if (EX[i] == sx && EY[i] == -1) ib = i;
                    R mx = R(0.0), my = R(0.0);
                    for (int i = 0; i < Q; ++i) {
                        if (i == ia || i == ib) continue;
                        mx += R((double)EX[i]) * f[i][n];
                        my += R((double)EY[i]) * f[i][n];
                    }
                    const R sum_ab = R((double)sx) * (jx - mx), diff_ab = jy - my;
                    f[ia][n] = R(0.5) * (sum_ab + diff_ab);
                    f[ib][n] = R(0.5) * (sum_ab - diff_ab);
                }
            }
        }
        // Stage 7b: wet-node walls -- the populations the wall nodes would receive from
        // beyond the wall, by non-equilibrium bounce-back with zero wall velocity (the
        // Zou-He closure; the momentum of the streamed populations is rho u - F / 2 with
        // the half-force shift, so zero velocity means -F / 2; reading A29).
        if (geo.ymode == MODE_WET) {
#pragma omp parallel for schedule(static)
            for (long long xx = 0; xx < (long long)nx; ++xx) {
                for (int y : {0, ny - 1}) {
                    const size_t n = (size_t)y * nx + (size_t)xx;
                    if (!fluid(n)) continue;
                    const R jx = R(-0.5) * Fx[n], jy = R(-0.5) * Fy[n];
                    const R d13 = f[1][n] - f[3][n];
                    if (y == 0) {  // unknown: directions with e_y = +1
                        f[2][n] = f[4][n] + R(2.0 / 3.0) * jy;
                        f[5][n] = f[7][n] - R(0.5) * d13 + R(1.0 / 6.0) * jy + R(0.5) * jx;
                        f[6][n] = f[8][n] + R(0.5) * d13 + R(1.0 / 6.0) * jy - R(0.5) * jx;
                    } else {  // unknown: directions with e_y = -1
                        f[4][n] = f[2][n] - R(2.0 / 3.0) * jy;
                        f[7][n] = f[5][n] + R(0.5) * d13 - R(1.0 / 6.0) * jy - R(0.5) * jx;
                        f[8][n] = f[6][n] - R(0.5) * d13 - R(1.0 / 6.0) * jy + R(0.5) * jx;
                    }
                }
            }
        }
        // Stage 8: conservative non-equilibrium bounce-back at every boundary node
        // (Sec. 3.3), with u(x_b, t+1) from the filled hydrodynamic populations
        // (reading A11); unknowns whose opposite is also unknown take the equilibrium
        // (reading A12).
#pragma omp parallel for schedule(static)
        for (long long nn = 0; nn < (long long)N; ++nn) {
            const size_t n = (size_t)nn;
            if (!fluid(n)) continue;
            const int x = (int)(n % nx), y = (int)(n / nx);
            bool unknown[Q];
            bool any = false;
            for (int i = 0; i < Q; ++i) {
                unknown[i] = geo.source(x, y, i).kind == SRC_SOLID;
                any = any || unknown[i];
            }
            if (!any) continue;
            R r = R(0.0), jx = R(0.0), jy = R(0.0);
            for (int i = 0; i < Q; ++i) {
                r += f[i][n];
                jx += R((double)EX[i]) * f[i][n];
                jy += R((double)EY[i]) * f[i][n];
            }
            R ubx = (jx + R(0.5) * Fx[n]) / r;
            R uby = (jy + R(0.5) * Fy[n]) / r;
            if (geo.wet_row(y)) ubx = uby = R(0.0);  // wall node: the wall velocity
            if (flags & FLAG_CNEBB_UB_ZERO) ubx = uby = R(0.0);
            for (int k = 0; k < 3; ++k) {
                // phi(x_b, t+1): known post-streaming populations plus the post-collision
                // populations that moved toward the solid.
                R phib = R(0.0);
                for (int i = 0; i < Q; ++i) phib += g[k][i][n];
                R known[Q];
                for (int i = 0; i < Q; ++i) known[i] = g[k][i][n];
                for (int i = 1; i < Q; ++i) {
                    if (!unknown[i]) continue;
                    const int o = OPP[i];
                    // (known[o] of an unknown o holds the post-collision population that
                    // left toward the solid in direction i: the alternative reading A12)
                    if (!unknown[o] || (flags & FLAG_CNEBB_PAIR_NEQ))
                        g[k][i][n] = geq(i, phib, ubx, uby) + (known[o] - geq(o, phib, ubx, uby));
                    else
                        g[k][i][n] = geq(i, phib, ubx, uby);
                }
                R rest = phib;
                for (int i = 1; i < Q; ++i) rest -= g[k][i][n];
                g[k][0][n] = rest;
            }
        }
        // Stage 9: history for the backward difference of F~ (Sec. 3.2).
        for (size_t n = 0; n < N; ++n) {
            if (!fluid(n)) continue;
            for (int k = 0; k < 3; ++k) Sprev[k][n] = Snew[k][n];
            uxp[n] = ux[n];
            uyp[n] = uy[n];
        }
        first = false;
        ++step;
    }

    // Momentum-exchange force on the solid (Sec. 4.3): over the fluid nodes x_f next
    // to a solid and the directions i pointing into it (x_f + e_i solid),
    // sum e_i (f_i^post(x_f, t) + f_opp(i)(x_f, t + 1)), with the post-collision values
    // of the last step and the populations it streamed and filled.  circle >= 0 keeps
    // the links into that circle only; circle < 0 keeps every solid (walls included).
    void drag(int circle, double out[2]) const {
        double fx = 0.0, fy = 0.0;
        for (size_t n = 0; n < N; ++n) {
            if (!fluid(n)) continue;
            const int x = (int)(n % nx), y = (int)(n / nx);
            for (int i = 1; i < Q; ++i) {
                const Src s = geo.source(x, y, OPP[i]);  // x - e_opp(i) = x + e_i
                if (s.kind != SRC_SOLID) continue;
                if (circle >= 0 && (s.node < 0 || geo.circle_of[s.node] != circle)) continue;
                const double v = val(fp[i][n]) + val(f[OPP[i]][n]);
                fx += (double)EX[i] * v;
                fy += (double)EY[i] * v;
            }
        }
        out[0] = fx;
        out[1] = fy;
    }
};

template <class R>
R mk(double v, double d);
template <>
double mk<double>(double v, double) { return v; }
template <>
Dual mk<Dual>(double v, double d) { return Dual(v, d); }

struct Handle {
    int dual = 0;
    Sim<double> sd;
    Sim<Dual> sx;
    Geometry& geo() { return dual ? sx.geo : sd.geo; }
};

template <class R>
void set_params(Sim<R>& s, double nu_s, double eta_p, double lam, double kappa,
                double Lambda_s, double Lambda_p, double dlam, double deta, int flags) {
    // mu_s = rho c_s^2 (tau_s1 - 1/2) with rho0 = 1 (reading A18), Lambda_s relation,
    // kappa = (tau_p1 - 1/2) c_s^2 and the tau_p2 relation (Sec. 3.1-3.2).
    const double ts1 = nu_s / CS2 + 0.5;
    const double ts2 = Lambda_s / (ts1 - 0.5) + 0.5;
    const double tp1 = kappa / CS2 + 0.5;
    const double tp2 = Lambda_p / (tp1 - 0.5) + 0.5;
    s.p.tau_s1 = R(ts1);
    s.p.tau_s2 = R(ts2);
    s.p.tau_p1 = R(tp1);
    s.p.tau_p2 = R(tp2);
    s.p.lam = mk<R>(lam, dlam);
    s.p.eta_p = mk<R>(eta_p, deta);
    s.flags = flags;
}

template <class R>
void init_state(Sim<R>& s, const double* rho0, const double* ux0, const double* uy0,
                const double* a0[3]) {
    const double phi0[3] = {1.0, 0.0, 1.0};
    for (size_t n = 0; n < s.N; ++n) {
        if (!s.fluid(n)) {
            for (int i = 0; i < Q; ++i) {
                s.f[i][n] = R(0.0);
                for (int k = 0; k < 3; ++k) s.g[k][i][n] = R(0.0);
            }
            continue;
        }
        const R r = R(rho0 ? rho0[n] : 1.0);
        const R vx = R(ux0 ? ux0[n] : 0.0), vy = R(uy0 ? uy0[n] : 0.0);
        for (int i = 0; i < Q; ++i) s.f[i][n] = feq(i, r, vx, vy);
        for (int k = 0; k < 3; ++k) {
            const R phi = R(a0[k] ? a0[k][n] : phi0[k]);
            for (int i = 0; i < Q; ++i) s.g[k][i][n] = geq(i, phi, vx, vy);
        }
        for (int k = 0; k < 3; ++k) s.Sprev[k][n] = R(0.0);
        s.uxp[n] = R(0.0);
        s.uyp[n] = R(0.0);
    }
    s.first = true;
    s.step = 0;
}

template <class R>
void read_fields(Sim<R>& s, double* out[6], double* tang[6]) {
    s.macros();
    for (size_t n = 0; n < s.N; ++n) {
        const bool fl = s.fluid(n);
        const R v[6] = {s.rho[n], s.ux[n], s.uy[n], s.A[0][n], s.A[1][n], s.A[2][n]};
        for (int c = 0; c < 6; ++c) {
            if (out && out[c]) out[c][n] = fl ? val(v[c]) : 0.0;
            if (tang && tang[c]) tang[c][n] = fl ? tan_(v[c]) : 0.0;
        }
    }
}

}  // namespace

extern "C" {

void* orc_create(int nx, int ny, int xmode, int ymode, const uint8_t* mask,
                 const double* circles, int ncircles, int dual) {
    if (nx < 1 || ny < 1 || xmode < 0 || xmode > 2 || ymode < 0 || ymode > 3 || ymode == 2)
        return nullptr;
    if (ymode == MODE_WET && ny < 5) return nullptr;
    Handle* h = new Handle();
    h->dual = dual;
    auto setup = [&](auto& s) {
        s.nx = nx; s.ny = ny;
        s.geo.build(nx, ny, xmode, ymode, mask, circles, ncircles);
        s.alloc();
        // wet-node walls: the wall rows and the two rows next to each (the one-sided
        // differences at the wall nodes) must be fluid
        bool ok = true;
        if (ymode == MODE_WET)
            for (int y : {0, 1, 2, ny - 3, ny - 2, ny - 1})
                for (int x = 0; x < nx; ++x) ok = ok && !s.geo.solid[(size_t)y * nx + x];
        return ok;
    };
    const bool ok = dual ? setup(h->sx) : setup(h->sd);
    if (!ok) {
        delete h;
        return nullptr;
    }
    return h;
}

void orc_destroy(void* hp) { delete static_cast<Handle*>(hp); }

void orc_set_threads(int n) {
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

int orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int orc_set_params(void* hp, double nu_s, double eta_p, double lam, double kappa,
                   double Lambda_s, double Lambda_p, int flags) {
    Handle* h = static_cast<Handle*>(hp);
    if (nu_s <= 0 || lam <= 0 || kappa <= 0 || Lambda_s <= 0 || Lambda_p <= 0 || eta_p < 0)
        return -1;
    if (h->dual) set_params(h->sx, nu_s, eta_p, lam, kappa, Lambda_s, Lambda_p, 0, 0, flags);
    else set_params(h->sd, nu_s, eta_p, lam, kappa, Lambda_s, Lambda_p, 0, 0, flags);
    return 0;
}

// Constitutive closure (MODEL_*) and its parameter: Giesekus alpha in [0, 1], PTT
// epsilon >= 0, FENE-P L^2 > 2; ignored for Oldroyd-B.
int orc_set_model(void* hp, int model, double mpar) {
    Handle* h = static_cast<Handle*>(hp);
    if (model < MODEL_OLDROYD_B || model > MODEL_FENE_P) return -1;
    if (model == MODEL_GIESEKUS && !(mpar >= 0.0 && mpar <= 1.0)) return -1;
    if ((model == MODEL_LPTT || model == MODEL_EPTT) && !(mpar >= 0.0)) return -1;
    if (model == MODEL_FENE_P && !(mpar > 2.0)) return -1;
    if (model == MODEL_OLDROYD_B) mpar = 0.0;
    if (h->dual) { h->sx.model = model; h->sx.mpar = mpar; }
    else { h->sd.model = model; h->sd.mpar = mpar; }
    return 0;
}

// Uniform force when fx/fy are null (values fx0, fy0).
int orc_set_force(void* hp, double fx0, double fy0, const double* fx, const double* fy) {
    Handle* h = static_cast<Handle*>(hp);
    auto doit = [&](auto& s) {
        using R = typename std::decay<decltype(s.Fx[0])>::type;
        for (size_t n = 0; n < s.N; ++n) {
            const double vx = fx ? fx[n] : fx0, vy = fy ? fy[n] : fy0;
            s.Fx[n] = mk<R>(vx, tan_(s.Fx[n]));
            s.Fy[n] = mk<R>(vy, tan_(s.Fy[n]));
        }
    };
    if (h->dual) doit(h->sx); else doit(h->sd);
    return 0;
}

// Tangent direction of the dual-number run: d lambda, d eta_p, d F(x) (nullable).
int orc_set_tangent(void* hp, double dlam, double deta, const double* dfx, const double* dfy) {
    Handle* h = static_cast<Handle*>(hp);
    if (!h->dual) return -1;
    Sim<Dual>& s = h->sx;
    s.p.lam.d = dlam;
    s.p.eta_p.d = deta;
    for (size_t n = 0; n < s.N; ++n) {
        s.Fx[n].d = dfx ? dfx[n] : 0.0;
        s.Fy[n].d = dfy ? dfy[n] : 0.0;
    }
    return 0;
}

int orc_set_inlet(void* hp, const double* ux, const double* axx, const double* axy,
                  const double* ayy) {
    Handle* h = static_cast<Handle*>(hp);
    auto doit = [&](auto& s) {
        using R = typename std::decay<decltype(s.Fx[0])>::type;
        for (int y = 0; y < s.ny; ++y) {
            s.uin[y] = R(ux[y]);
            s.ain[0][y] = R(axx[y]);
            s.ain[1][y] = R(axy[y]);
            s.ain[2][y] = R(ayy[y]);
        }
    };
    if (h->dual) doit(h->sx); else doit(h->sd);
    return 0;
}

// Equilibrium initial state (f = f^eq(rho0, u0), g = g^eq(A0, u0)); null arrays take
// rho = 1, u = 0, A = I.
int orc_init(void* hp, const double* rho, const double* ux, const double* uy,
             const double* axx, const double* axy, const double* ayy) {
    Handle* h = static_cast<Handle*>(hp);
    const double* a0[3] = {axx, axy, ayy};
    if (h->dual) init_state(h->sx, rho, ux, uy, a0); else init_state(h->sd, rho, ux, uy, a0);
    return 0;
}

int orc_step(void* hp, long long nsteps) {
    Handle* h = static_cast<Handle*>(hp);
    for (long long t = 0; t < nsteps; ++t) {
        if (h->dual) h->sx.step_once(); else h->sd.step_once();
    }
    return 0;
}

long long orc_get_step(void* hp) {
    Handle* h = static_cast<Handle*>(hp);
    return h->dual ? h->sx.step : h->sd.step;
}

// Macroscopic fields at the current time (rho, ux, uy, Axx, Axy, Ayy), 0 on solids.
int orc_read(void* hp, double* rho, double* ux, double* uy, double* axx, double* axy,
             double* ayy) {
    Handle* h = static_cast<Handle*>(hp);
    double* out[6] = {rho, ux, uy, axx, axy, ayy};
    if (h->dual) read_fields(h->sx, out, nullptr); else read_fields(h->sd, out, nullptr);
    return 0;
}

int orc_read_tangent(void* hp, double* rho, double* ux, double* uy, double* axx,
                     double* axy, double* ayy) {
    Handle* h = static_cast<Handle*>(hp);
    if (!h->dual) return -1;
    double* t[6] = {rho, ux, uy, axx, axy, ayy};
    read_fields(h->sx, nullptr, t);
    return 0;
}

// History used by the next step: S_prev (3 components) and u_prev, and the first-step flag.
int orc_read_history(void* hp, double* sxx, double* sxy, double* syy, double* uxp,
                     double* uyp) {
    Handle* h = static_cast<Handle*>(hp);
    auto doit = [&](auto& s) {
        double* o[5] = {sxx, sxy, syy, uxp, uyp};
        for (size_t n = 0; n < s.N; ++n) {
            const double v[5] = {val(s.Sprev[0][n]), val(s.Sprev[1][n]), val(s.Sprev[2][n]),
                                 val(s.uxp[n]), val(s.uyp[n])};
            for (int c = 0; c < 5; ++c)
                if (o[c]) o[c][n] = v[c];
        }
        return s.first ? 1 : 0;
    };
    return h->dual ? doit(h->sx) : doit(h->sd);
}

// Momentum-exchange force on circle `circle` (all solids if < 0) after the last step;
// -1 before the first step.
int orc_drag(void* hp, int circle, double* out2) {
    Handle* h = static_cast<Handle*>(hp);
    if (h->dual ? h->sx.first : h->sd.first) return -1;
    if (h->dual) h->sx.drag(circle, out2);
    else h->sd.drag(circle, out2);
    return 0;
}

// Raw populations at the current time (post-stream, post-boundary): f[9][N], g[3][9][N].
int orc_read_populations(void* hp, double* f, double* g) {
    Handle* h = static_cast<Handle*>(hp);
    if (h->dual) return -1;
    Sim<double>& s = h->sd;
    for (int i = 0; i < Q; ++i)
        for (size_t n = 0; n < s.N; ++n) {
            if (f) f[(size_t)i * s.N + n] = s.f[i][n];
            for (int k = 0; k < 3; ++k)
                if (g) g[((size_t)k * Q + i) * s.N + n] = s.g[k][i][n];
        }
    return 0;
}

// Node classes (0 fluid, 1 solid, 2 fluid boundary node) and the boundary-link list:
// one entry per fluid node and direction d (1..8) with x + e_d solid, as (node index
// y*nx + x, d, q), sorted by (node, d).  Returns the number of links; writes at most
// cap entries (pass cap = 0 to query).
int orc_geometry(void* hp, uint8_t* cls, int32_t* lnode, int8_t* ldir, double* lq, int cap) {
    Handle* h = static_cast<Handle*>(hp);
    Geometry& geo = h->geo();
    int cnt = 0;
    for (int y = 0; y < geo.ny; ++y)
        for (int x = 0; x < geo.nx; ++x) {
            const int n = y * geo.nx + x;
            if (geo.solid[n]) { if (cls) cls[n] = 1; continue; }
            bool b = false;
            for (int d = 1; d < Q; ++d) {
                // the link toward the solid in direction d is the source of direction OPP[d]
                const Src s = geo.source(x, y, OPP[d]);
                if (s.kind != SRC_SOLID) continue;
                b = true;
                if (cnt < cap) {
                    lnode[cnt] = n;
                    ldir[cnt] = (int8_t)d;
                    lq[cnt] = s.q;
                }
                ++cnt;
            }
            if (cls) cls[n] = b ? 2 : 0;
        }
    return cnt;
}

// Lattice tables for tests: e_x, e_y, opposite (each 9 ints).
void orc_lattice(int* ex, int* ey, int* opp, double* w) {
    for (int i = 0; i < Q; ++i) { ex[i] = EX[i]; ey[i] = EY[i]; opp[i] = OPP[i]; w[i] = W[i]; }
}

// Single-node pieces for identity checks (double only).
void orc_node_feq(double rho, double ux, double uy, double* out9) {
    for (int i = 0; i < Q; ++i) out9[i] = feq(i, rho, ux, uy);
}
void orc_node_geq(double phi, double ux, double uy, double* out9) {
    for (int i = 0; i < Q; ++i) out9[i] = geq(i, phi, ux, uy);
}
void orc_node_hydro(const double* f9, double Fx, double Fy, double tau_s1, double tau_s2,
                    double txx, double txy, double tyy, double Dx, double Dy, double* out9) {
    double r = 0, jx = 0, jy = 0;
    for (int i = 0; i < Q; ++i) { r += f9[i]; jx += EX[i] * f9[i]; jy += EY[i] * f9[i]; }
    const double ux = (jx + 0.5 * Fx) / r, uy = (jy + 0.5 * Fy) / r;
    Relax<double> p{tau_s1, tau_s2, 1.0, 1.0, 1.0, 0.0};
    const double tau_ab[2][2] = {{txx, txy}, {txy, tyy}};
    collide_hydro(f9, r, ux, uy, Fx, Fy, tau_ab, Dx, Dy, p, out9);
}
void orc_node_cde(const double* g9, double rho, double ux, double uy, double Fx, double Fy,
                  double S, double Sp, double uxp, double uyp, double tau_p1, double tau_p2,
                  double* out9) {
    double phi = 0;
    for (int i = 0; i < Q; ++i) phi += g9[i];
    Relax<double> p{1.0, 1.0, tau_p1, tau_p2, 1.0, 0.0};
    collide_cde(g9, phi, rho, ux, uy, Fx, Fy, S, Sp, uxp, uyp, p, out9);
}
void orc_node_source_model(const double* A3, const double* L4, double lam, int model,
                           double mpar, double* S3) {
    const double A[2][2] = {{A3[0], A3[1]}, {A3[1], A3[2]}};
    const double L[2][2] = {{L4[0], L4[1]}, {L4[2], L4[3]}};
    double S[2][2];
    constitutive_source(A, L, lam, model, mpar, S);
    S3[0] = S[0][0]; S3[1] = S[0][1]; S3[2] = S[1][1];
}
void orc_node_source(const double* A3, const double* L4, double lam, double* S3) {
    orc_node_source_model(A3, L4, lam, MODEL_OLDROYD_B, 0.0, S3);
}
double orc_node_fd(int lo_solid, double qlo, double plo, double p0, int hi_solid, double qhi,
                   double phi) {
    return fd_axis(lo_solid != 0, qlo, plo, p0, hi_solid != 0, qhi, phi);
}

}  // extern "C"
