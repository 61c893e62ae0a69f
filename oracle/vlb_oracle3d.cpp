/*
 * vlb_oracle3d.cpp -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, double-precision CPU implementation of the coupled viscoelastic
 * lattice Boltzmann step of arXiv:2508.16997 extended to three dimensions on the D3Q19
 * or the D3Q27 lattice (the paper works in two dimensions and calls the
 * three-dimensional extension straightforward, Sec. 3.1; the readings of that extension
 * are listed in the design notes under A32).  Only the tests and the CPU-baseline leg of the benchmark may load
 * it; it shares no code with the HIP library nor with the two-dimensional oracle.
 *
 * Same stages and the same formulas as the two-dimensional method, with every tensor
 * index running over x, y, z:
 *   1. rho and u with the half-force shift                               (Sec. 3.1)
 *   2. conformation A (six components, one convection-diffusion lattice each) and the
 *      polymer stress (eta_p / lambda) F_s(A) of the closure (Oldroyd-B: A - I) (Sec. 2.2-2.3)
 *   3. velocity gradient L[g][b] = d_g u_b and D_a = d_a(rho u_a^3) by central
 *      differences; next to a flat half-way wall the quadratic through the no-slip wall
 *      value half a spacing away                                         (readings A6/A7)
 *   4. constitutive source Phi = -F_r(A)/lambda + A L + (A L)^T + A tr L  (Sec. 3.2)
 *   5. hydrodynamic TRT regularized collision: Hermite moments of orders 0..3 of f - f^eq
 *      (third order on the lattice's own orthogonal basis and norms), tau_s1 on orders 0..2,
 *      tau_s2 on order 3, plus G_i (diagonal third-order defects D_a), F_i and T_i
 *                                                                         (Sec. 3.1)
 *   6. six convection-diffusion TRT regularized collisions with the auxiliary term
 *      G~_i, the source term F~_i and half its backward time difference   (Sec. 3.2)
 *   7. streaming (pull) with half-way bounce-back of f at flat walls normal to y and at
 *      the faces of solid nodes; the
 *      conformation populations that left toward the wall are the CNEBB input
 *   8. conservative non-equilibrium bounce-back for every conformation lattice at
 *      wall-adjacent nodes                                                (Sec. 3.3)
 *   9. history of S and u for the time difference
 *
 * Axes x and z are periodic; y is periodic or bounded by half-way walls; any node may be
 * solid (a staircase obstacle, read out at rest).  Uniform body
 * force.  Index convention of fields: [z][y][x], x fastest.
 *
 * Build: g++ -O2 -std=c++17 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math).
 */
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ----------------------------------------------------------------------------------
// D3Q19: the rest velocity, the six axis velocities (weight 1/18) and the twelve face
// diagonals (weight 1/36), enumerated from {-1, 0, 1}^3 with |e|^2 <= 2.
// D3Q27: all of {-1, 0, 1}^3, the tensor product of D1Q3 (weights 2/3, 1/6, 1/6): rest
// 8/27, axis 2/27, face diagonals 1/54, corners 1/216.  c_s^2 = 1/3 on both.
// ----------------------------------------------------------------------------------
const int QMAX = 27;
const int NB3MAX = 7;
const double CS2 = 1.0 / 3.0;

inline double kd(int a, int b) { return a == b ? 1.0 : 0.0; }

// A third-order basis function: a sum of coef * H_abc terms.
struct Term {
    double coef;
    int a, b, c;
};
struct Basis3 {
    int nterms;
    Term t[2];
};

struct Lattice {
    int Q;
    int E[QMAX][3], OPP[QMAX];
    double W[QMAX];
    int nb3;
    Basis3 b3[NB3MAX];
    double norm3[NB3MAX];  // lattice norms sum_i w_i h_m(e_i)^2

    double ec(int i, int a) const { return (double)E[i][a]; }
    // Hermite polynomials of orders 1..3 (Sec. 3.1), indices over x, y, z.
    double H1(int i, int a) const { return ec(i, a); }
    double H2(int i, int a, int b) const { return ec(i, a) * ec(i, b) - CS2 * kd(a, b); }
    double H3(int i, int a, int b, int c) const {
        return ec(i, a) * ec(i, b) * ec(i, c) -
               CS2 * (ec(i, a) * kd(b, c) + ec(i, b) * kd(a, c) + ec(i, c) * kd(a, b));
    }
    double h3(int i, int m) const {
        double v = 0.0;
        for (int k = 0; k < b3[m].nterms; ++k) v += b3[m].t[k].coef * H3(i, b3[m].t[k].a, b3[m].t[k].b, b3[m].t[k].c);
        return v;
    }
    // the matching third-order moment of the continuous equilibrium per unit density
    double u3(const double u[3], int m) const {
        double v = 0.0;
        for (int k = 0; k < b3[m].nterms; ++k) v += b3[m].t[k].coef * u[b3[m].t[k].a] * u[b3[m].t[k].b] * u[b3[m].t[k].c];
        return v;
    }
    bool rest(int i) const { return E[i][0] == 0 && E[i][1] == 0 && E[i][2] == 0; }

    explicit Lattice(int q) : Q(q) {
        int n = 0;
        for (int norm = 0; norm <= (q == 27 ? 3 : 2); ++norm)
            for (int a = -1; a <= 1; ++a)
                for (int b = -1; b <= 1; ++b)
                    for (int c = -1; c <= 1; ++c)
                        if (a * a + b * b + c * c == norm) {
                            E[n][0] = a;
                            E[n][1] = b;
                            E[n][2] = c;
                            if (q == 27) {
                                const double w1[2] = {2.0 / 3.0, 1.0 / 6.0};
                                W[n] = w1[a * a] * w1[b * b] * w1[c * c];
                            } else {
                                W[n] = norm == 0 ? 1.0 / 3.0 : (norm == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
                            }
                            ++n;
                        }
        for (int i = 0; i < Q; ++i)
            for (int j = 0; j < Q; ++j)
                if (E[j][0] == -E[i][0] && E[j][1] == -E[i][1] && E[j][2] == -E[i][2]) OPP[i] = j;
        // Third-order content (reading A32).  No H_aaa survives on either lattice.
        // D3Q19: H_xyz vanishes at every velocity; the six xxy-type polynomials remain but
        // are neither orthogonal nor of their continuous norm 2 c_s^6, so the basis is the
        // six combinations h_{c,s} = H_aab + s H_bcc (s = +1, -1) for (a, b, c) = (x, y, z),
        // (z, x, y), (y, z, x) -- H_xxy -+ H_yzz, H_zzx -+ H_xyy, H_yyz -+ H_zxx -- mutually
        // orthogonal on D3Q19 with lattice norms 2 c_s^6 (s = +1) and 6 c_s^6 (s = -1).
        // D3Q27: the six H_aab and H_xyz themselves, orthogonal with their continuous norms
        // 2 c_s^6 and c_s^6 (products of one-dimensional Hermite polynomials).
        const int HC[3][3] = {{0, 1, 2}, {2, 0, 1}, {1, 2, 0}};
        nb3 = 0;
        if (q == 19) {
            for (int c = 0; c < 3; ++c)
                for (int sg = 1; sg >= -1; sg -= 2) {
                    const int a = HC[c][0], b = HC[c][1], d = HC[c][2];
                    b3[nb3].nterms = 2;
                    b3[nb3].t[0] = {1.0, a, a, b};
                    b3[nb3].t[1] = {(double)sg, b, d, d};
                    ++nb3;
                }
        } else {
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b)
                    if (a != b) {
                        b3[nb3].nterms = 1;
                        b3[nb3].t[0] = {1.0, a, a, b};
                        ++nb3;
                    }
            b3[nb3].nterms = 1;
            b3[nb3].t[0] = {1.0, 0, 1, 2};
            ++nb3;
        }
        for (int m = 0; m < nb3; ++m) {
            double s = 0.0;
            for (int i = 0; i < Q; ++i) s += W[i] * h3(i, m) * h3(i, m);
            norm3[m] = s;
        }
    }
};
const Lattice LAT19(19), LAT27(27);

// Hydrodynamic equilibrium, Hermite expansion to third order (Sec. 3.1); the third
// order expanded in the lattice's third-order basis with its lattice norms, so that the
// lattice equilibrium has the continuous third-order moments along every direction the
// lattice resolves.
double feq(const Lattice& L, int i, double rho, const double u[3]) {
    double s = 1.0;
    for (int a = 0; a < 3; ++a) s += L.H1(i, a) / CS2 * u[a];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) s += L.H2(i, a, b) / (2.0 * CS2 * CS2) * u[a] * u[b];
    for (int m = 0; m < L.nb3; ++m) s += L.h3(i, m) / L.norm3[m] * L.u3(u, m);
    return L.W[i] * rho * s;
}

// Convection-diffusion equilibrium, second-order Hermite expansion (Sec. 3.2).
double geq(const Lattice& L, int i, double phi, const double u[3]) {
    double s = 1.0;
    for (int a = 0; a < 3; ++a) s += L.H1(i, a) / CS2 * u[a];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) s += L.H2(i, a, b) / (2.0 * CS2 * CS2) * u[a] * u[b];
    return L.W[i] * phi * s;
}

struct Params {
    double tau_s1 = 1.0, tau_s2 = 1.0, tau_p1 = 1.0, tau_p2 = 1.0, lam = 1.0, eta_p = 0.0;
    double F[3] = {0.0, 0.0, 0.0};
    int no_source = 0;
    int model = 0;      // constitutive closure (MODEL_*) and its parameter
    double mpar = 0.0;
};

// Constitutive closures (Sec. 2.2, the model function F(A)) in conformation form with the
// three-dimensional trace (tr A = 3 at rest), B = A - I: relaxation function F_r in the
// conformation equation, stress function F_s in the Kramers relation (reading A28 with
// every index over x, y, z):
//   Oldroyd-B  F_r = F_s = B
//   Giesekus   F_r = B + alpha B B, F_s = B                 (mpar = alpha)
//   PTT        F_r = Y B, Y = 1 + eps (tr A - 3) (linear) or exp(eps (tr A - 3)), F_s = B
//   FENE-P     F_r = F_s = f A - I, f = (L^2 - 3) / (L^2 - tr A)   (mpar = L^2)
enum { MODEL_OLDROYD_B = 0, MODEL_GIESEKUS = 1, MODEL_LPTT = 2, MODEL_EPTT = 3, MODEL_FENE_P = 4 };
void model_functions3(const double A[3][3], int model, double mp, double Fr[3][3],
                      double Fs[3][3]) {
    double B[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) B[a][b] = A[a][b] - kd(a, b);
    const double tr = A[0][0] + A[1][1] + A[2][2];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            Fr[a][b] = B[a][b];
            Fs[a][b] = B[a][b];
        }
    if (model == MODEL_GIESEKUS) {
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double bb = 0.0;
                for (int c = 0; c < 3; ++c) bb += B[a][c] * B[c][b];
                Fr[a][b] += mp * bb;
            }
    } else if (model == MODEL_LPTT || model == MODEL_EPTT) {
        const double x = mp * (tr - 3.0);
        const double Y = model == MODEL_LPTT ? 1.0 + x : std::exp(x);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) Fr[a][b] = Y * B[a][b];
    } else if (model == MODEL_FENE_P) {
        const double f = (mp - 3.0) / (mp - tr);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                Fr[a][b] = f * A[a][b] - kd(a, b);
                Fs[a][b] = Fr[a][b];
            }
    }
}

// Hydrodynamic TRT regularized collision (Sec. 3.1, three-dimensional indices).
void collide_hydro(const Lattice& L, const double* f, double rho, const double u[3],
                   const double F[3], const double tau[3][3], const double D[3], const Params& p,
                   double* out) {
    const int Q = L.Q;
    double fe[QMAX];
    for (int i = 0; i < Q; ++i) fe[i] = feq(L, i, rho, u);
    double A0 = 0.0, A1[3] = {0.0, 0.0, 0.0}, A2[3][3], A3[NB3MAX];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) A2[a][b] = 0.0;
    for (int m = 0; m < L.nb3; ++m) A3[m] = 0.0;
    for (int i = 0; i < Q; ++i) {
        const double d = f[i] - fe[i];
        A0 += d;
        for (int a = 0; a < 3; ++a) A1[a] += L.H1(i, a) * d;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) A2[a][b] += L.H2(i, a, b) * d;
        for (int m = 0; m < L.nb3; ++m) A3[m] += L.h3(i, m) * d;
    }
    const double c1 = 1.0 - 1.0 / p.tau_s1, c2 = 1.0 - 1.0 / p.tau_s2;
    const double h1 = 1.0 - 1.0 / (2.0 * p.tau_s1);
    for (int i = 0; i < Q; ++i) {
        double reg1 = A0;
        for (int a = 0; a < 3; ++a) reg1 += L.H1(i, a) / CS2 * A1[a];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) reg1 += L.H2(i, a, b) / (2.0 * CS2 * CS2) * A2[a][b];
        double reg2 = 0.0;  // projection on the third-order basis with its lattice norms
        for (int m = 0; m < L.nb3; ++m) reg2 += L.h3(i, m) / L.norm3[m] * A3[m];
        // G_i: d_g Phi_abg restricted to the diagonal defects (a, a) <- d_a(rho u_a^3)
        double sumG = 0.0, sumT = 0.0, sumF = 0.0;
        for (int a = 0; a < 3; ++a) sumG += L.H2(i, a, a) / (6.0 * CS2 * CS2 * CS2) * D[a];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) sumT += L.H2(i, a, b) / (2.0 * CS2 * CS2) * tau[a][b];
        for (int a = 0; a < 3; ++a) sumF += L.H1(i, a) / CS2 * F[a];
        const double Gi = -L.W[i] * h1 * sumG;
        const double Ti = -L.W[i] * sumT / p.tau_s1;
        const double Fi = h1 * L.W[i] * sumF;
        out[i] = fe[i] + L.W[i] * c1 * reg1 + L.W[i] * c2 * reg2 + Gi + Fi + Ti;
    }
}

// Convection-diffusion TRT regularized collision for one component (Sec. 3.2).
void collide_cde(const Lattice& L, const double* g, double phi, double rho, const double u[3],
                 const double F[3], double S, double Sp, const double up[3], const Params& p,
                 double* out) {
    const int Q = L.Q;
    double ge[QMAX];
    for (int i = 0; i < Q; ++i) ge[i] = geq(L, i, phi, u);
    double B0 = 0.0, B1[3] = {0.0, 0.0, 0.0}, B2[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) B2[a][b] = 0.0;
    for (int i = 0; i < Q; ++i) {
        const double d = g[i] - ge[i];
        B0 += d;
        for (int a = 0; a < 3; ++a) B1[a] += L.H1(i, a) * d;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) B2[a][b] += L.H2(i, a, b) * d;
    }
    const double c1 = 1.0 - 1.0 / p.tau_p1, c2 = 1.0 - 1.0 / p.tau_p2;
    const double h2 = 1.0 - 1.0 / (2.0 * p.tau_p1);
    for (int i = 0; i < Q; ++i) {
        double reg1 = B0;
        for (int a = 0; a < 3; ++a) reg1 += L.H1(i, a) / CS2 * B1[a];
        double reg2 = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) reg2 += L.H2(i, a, b) / (2.0 * CS2 * CS2) * B2[a][b];
        double eF = 0.0, eu = 0.0, eup = 0.0;
        for (int a = 0; a < 3; ++a) {
            eF += L.ec(i, a) / CS2 * F[a];
            eu += L.ec(i, a) / CS2 * u[a];
            eup += L.ec(i, a) / CS2 * up[a];
        }
        const double W = L.W[i];
        const double Gt = W * h2 * eF * phi / rho;
        const double Ft_now = W * S + h2 * W * eu * S;
        const double Ft_prev = W * Sp + h2 * W * eup * Sp;
        out[i] = ge[i] + W * c1 * reg1 + W * c2 * reg2 + Gt + Ft_now +
                 0.5 * (Ft_now - Ft_prev);
    }
}

// Components of the symmetric conformation tensor, one lattice each.
const int KA[6] = {0, 0, 0, 1, 1, 2}, KB[6] = {0, 1, 2, 1, 2, 2};
inline int comp(int a, int b) {
    if (a > b) std::swap(a, b);
    for (int k = 0; k < 6; ++k)
        if (KA[k] == a && KB[k] == b) return k;
    return -1;
}

// Central difference along one axis, or (flat half-way wall half a spacing away) the
// quadratic through the no-slip wall value 0 (reading A6 with q = 1/2).
double fd(bool lo_wall, double vlo, double v0, bool hi_wall, double vhi) {
    const double q = 0.5;
    if (!lo_wall && !hi_wall) return 0.5 * (vhi - vlo);
    if (lo_wall && !hi_wall) return q / (1.0 + q) * vhi + (1.0 - q) / q * v0;
    if (!lo_wall) return -(q / (1.0 + q) * vlo + (1.0 - q) / q * v0);
    return 0.0;
}

// Constitutive source of the conformation equation (Sec. 3.2, every index over x, y, z):
// Phi_ab = -F_r(A)_ab / lambda + sum_g (A_ag L_gb + A_gb L_ga) + A_ab tr L with
// L_gb = d_g u_b (F_r = A - I for Oldroyd-B).
void source3(const double Am[3][3], const double L[3][3], double lam, double S[3][3],
             int model = MODEL_OLDROYD_B, double mp = 0.0) {
    const double trL = L[0][0] + L[1][1] + L[2][2];
    double Fr[3][3], Fs[3][3];
    model_functions3(Am, model, mp, Fr, Fs);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = -Fr[a][b] / lam;
            for (int gm = 0; gm < 3; ++gm) s += Am[a][gm] * L[gm][b] + Am[gm][b] * L[gm][a];
            S[a][b] = s + Am[a][b] * trL;
        }
}

struct Sim {
    const Lattice& lat;
    int Q;
    int nx, ny, nz, ywall;
    size_t N;
    Params p;
    std::vector<double> f[QMAX], fp[QMAX], g[6][QMAX], gp[6][QMAX];
    std::vector<double> rho, u[3], A[6], Sprev[6], uprev[3];
    std::vector<uint8_t> solid;  // 1 = solid node (half-way bounce-back / CNEBB at its links)
    bool first = true;
    long long step = 0;

    Sim(const Lattice& lat_, int nx_, int ny_, int nz_, int ywall_)
        : lat(lat_), Q(lat_.Q), nx(nx_), ny(ny_), nz(nz_), ywall(ywall_) {
        N = (size_t)nx * ny * nz;
        for (int i = 0; i < Q; ++i) {
            f[i].assign(N, 0.0);
            fp[i].assign(N, 0.0);
            for (int k = 0; k < 6; ++k) {
                g[k][i].assign(N, 0.0);
                gp[k][i].assign(N, 0.0);
            }
        }
        rho.assign(N, 1.0);
        for (int a = 0; a < 3; ++a) {
            u[a].assign(N, 0.0);
            uprev[a].assign(N, 0.0);
        }
        for (int k = 0; k < 6; ++k) {
            A[k].assign(N, 0.0);
            Sprev[k].assign(N, 0.0);
        }
        solid.assign(N, 0);
    }
    size_t idx(int x, int y, int z) const { return ((size_t)z * ny + y) * nx + x; }
    static int wrap(int v, int n) { return ((v % n) + n) % n; }
    // Source node of the pull x - e_i: false when it lies beyond a wall or is solid (the
    // link then ends half way, at the wall or the solid node's face).
    bool source(int x, int y, int z, int i, size_t* s) const {
        int xs = wrap(x - lat.E[i][0], nx), ys = y - lat.E[i][1], zs = wrap(z - lat.E[i][2], nz);
        if (ys < 0 || ys >= ny) {
            if (ywall) return false;
            ys = wrap(ys, ny);
        }
        *s = idx(xs, ys, zs);
        return solid[*s] == 0;
    }

    void macros() {
        for (size_t n = 0; n < N; ++n) {
            if (solid[n]) {  // read out at rest
                rho[n] = 1.0;
                for (int a = 0; a < 3; ++a) u[a][n] = 0.0;
                for (int k = 0; k < 6; ++k) A[k][n] = KA[k] == KB[k] ? 1.0 : 0.0;
                continue;
            }
            double r = 0.0, j[3] = {0.0, 0.0, 0.0};
            for (int i = 0; i < Q; ++i) {
                r += f[i][n];
                for (int a = 0; a < 3; ++a) j[a] += lat.ec(i, a) * f[i][n];
            }
            rho[n] = r;
            for (int a = 0; a < 3; ++a) u[a][n] = (j[a] + 0.5 * p.F[a]) / r;
            for (int k = 0; k < 6; ++k) {
                double s = 0.0;
                for (int i = 0; i < Q; ++i) s += g[k][i][n];
                A[k][n] = s;
            }
        }
    }

    void init(const double* r0, const double* u0[3], const double* a0[6]) {
        for (size_t n = 0; n < N; ++n) {
            const double r = r0 ? r0[n] : 1.0;
            double v[3];
            for (int a = 0; a < 3; ++a) v[a] = u0[a] ? u0[a][n] : 0.0;
            for (int i = 0; i < Q; ++i) f[i][n] = feq(lat, i, r, v);
            for (int k = 0; k < 6; ++k) {
                const double phi = a0[k] ? a0[k][n] : (KA[k] == KB[k] ? 1.0 : 0.0);
                for (int i = 0; i < Q; ++i) g[k][i][n] = geq(lat, i, phi, v);
            }
        }
        first = true;
        step = 0;
    }

    void step_once() {
        macros();
        std::vector<double> Snew[6];
        for (int k = 0; k < 6; ++k) Snew[k].assign(N, 0.0);
#pragma omp parallel for schedule(static)
        for (long long nn = 0; nn < (long long)N; ++nn) {
            const size_t n = (size_t)nn;
            if (solid[n]) continue;
            const int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((size_t)nx * ny));
            // neighbours along the axes; a wall or a solid neighbour puts the no-slip value
            // half a spacing away (reading A6 with q = 1/2)
            const size_t nb[3][2] = {{idx(wrap(x - 1, nx), y, z), idx(wrap(x + 1, nx), y, z)},
                                     {idx(x, wrap(y - 1, ny), z), idx(x, wrap(y + 1, ny), z)},
                                     {idx(x, y, wrap(z - 1, nz)), idx(x, y, wrap(z + 1, nz))}};
            bool wl[3], wh[3];
            for (int ax = 0; ax < 3; ++ax) {
                wl[ax] = (ax == 1 && ywall && y == 0) || solid[nb[ax][0]];
                wh[ax] = (ax == 1 && ywall && y == ny - 1) || solid[nb[ax][1]];
            }
            auto dax = [&](int ax, auto val) {
                return fd(wl[ax], wl[ax] ? 0.0 : val(nb[ax][0]), val(n), wh[ax],
                          wh[ax] ? 0.0 : val(nb[ax][1]));
            };
            double L[3][3], D[3];
            for (int gm = 0; gm < 3; ++gm)
                for (int b = 0; b < 3; ++b) L[gm][b] = dax(gm, [&](size_t m) { return u[b][m]; });
            for (int a = 0; a < 3; ++a)
                D[a] = dax(a, [&](size_t m) { return rho[m] * u[a][m] * u[a][m] * u[a][m]; });
            double Am[3][3];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) Am[a][b] = A[comp(a, b)][n];
            // constitutive source (Oldroyd-B)
            double S[3][3];
            source3(Am, L, p.lam, S, p.model, p.mpar);
            if (p.no_source)
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) S[a][b] = 0.0;
            double tau[3][3], Fr[3][3], Fs[3][3];
            model_functions3(Am, p.model, p.mpar, Fr, Fs);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) tau[a][b] = p.eta_p / p.lam * Fs[a][b];
            double fl[QMAX], out[QMAX];
            for (int i = 0; i < Q; ++i) fl[i] = f[i][n];
            const double uu[3] = {u[0][n], u[1][n], u[2][n]};
            collide_hydro(lat, fl, rho[n], uu, p.F, tau, D, p, out);
            for (int i = 0; i < Q; ++i) fp[i][n] = out[i];
            const double upv[3] = {first ? uu[0] : uprev[0][n], first ? uu[1] : uprev[1][n],
                                   first ? uu[2] : uprev[2][n]};
            for (int k = 0; k < 6; ++k) {
                double gl[QMAX], go[QMAX];
                for (int i = 0; i < Q; ++i) gl[i] = g[k][i][n];
                const double Sk = S[KA[k]][KB[k]];
                const double Spk = first ? Sk : Sprev[k][n];
                collide_cde(lat, gl, A[k][n], rho[n], uu, p.F, Sk, Spk, upv, p, go);
                for (int i = 0; i < Q; ++i) gp[k][i][n] = go[i];
                Snew[k][n] = Sk;
            }
        }
        // streaming (pull), half-way bounce-back of f at the walls, wall-bound g kept
#pragma omp parallel for schedule(static)
        for (long long nn = 0; nn < (long long)N; ++nn) {
            const size_t n = (size_t)nn;
            if (solid[n]) continue;
            const int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((size_t)nx * ny));
            for (int i = 0; i < Q; ++i) {
                size_t s;
                if (source(x, y, z, i, &s)) {
                    f[i][n] = fp[i][s];
                    for (int k = 0; k < 6; ++k) g[k][i][n] = gp[k][i][s];
                } else {
                    f[i][n] = fp[lat.OPP[i]][n];
                    for (int k = 0; k < 6; ++k) g[k][i][n] = gp[k][lat.OPP[i]][n];
                }
            }
        }
        // CNEBB at wall-adjacent nodes (Sec. 3.3): phi_b = sum of the pulled populations
        // (known ones plus those that left toward the wall), unknowns rebuilt from the
        // equilibrium at (phi_b, u_b) plus the non-equilibrium part of the known
        // opposite, g_0 restores phi_b; u_b from the filled f with the half-force shift
        // (reading A11).
        {
#pragma omp parallel for schedule(static)
            for (long long nn = 0; nn < (long long)N; ++nn) {
                const size_t n = (size_t)nn;
                if (solid[n]) continue;
                const int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((size_t)nx * ny));
                bool unknown[QMAX], any = false;
                for (int i = 0; i < Q; ++i) {
                    size_t s;
                    unknown[i] = !source(x, y, z, i, &s);
                    any = any || unknown[i];
                }
                if (!any) continue;
                double r = 0.0, j[3] = {0.0, 0.0, 0.0};
                for (int i = 0; i < Q; ++i) {
                    r += f[i][n];
                    for (int a = 0; a < 3; ++a) j[a] += lat.ec(i, a) * f[i][n];
                }
                double ub[3];
                for (int a = 0; a < 3; ++a) ub[a] = (j[a] + 0.5 * p.F[a]) / r;
                for (int k = 0; k < 6; ++k) {
                    double gabs[QMAX], phib = 0.0;
                    for (int i = 0; i < Q; ++i) {
                        gabs[i] = g[k][i][n];
                        phib += gabs[i];
                    }
                    double known[QMAX];
                    for (int i = 0; i < Q; ++i) known[i] = gabs[i];
                    for (int i = 0; i < Q; ++i) {
                        if (!unknown[i]) continue;
                        const int o = lat.OPP[i];
                        gabs[i] = geq(lat, i, phib, ub);
                        if (!unknown[o]) gabs[i] += known[o] - geq(lat, o, phib, ub);
                    }
                    double rest = phib;
                    for (int i = 0; i < Q; ++i)
                        if (!lat.rest(i)) rest -= gabs[i];
                    for (int i = 0; i < Q; ++i)
                        if (lat.rest(i)) gabs[i] = rest;
                    for (int i = 0; i < Q; ++i) g[k][i][n] = gabs[i];
                }
            }
        }
        for (size_t n = 0; n < N; ++n) {
            for (int k = 0; k < 6; ++k) Sprev[k][n] = Snew[k][n];
            for (int a = 0; a < 3; ++a) uprev[a][n] = u[a][n];
        }
        first = false;
        ++step;
    }
};

}  // namespace

extern "C" {

// q: 19 (D3Q19) or 27 (D3Q27).
void* o3_create(int nx, int ny, int nz, int ywall, int q) {
    if (nx < 1 || ny < 1 || nz < 1 || (ywall && ny < 3) || (q != 19 && q != 27)) return nullptr;
    return new Sim(q == 27 ? LAT27 : LAT19, nx, ny, nz, ywall ? 1 : 0);
}
void o3_destroy(void* h) { delete static_cast<Sim*>(h); }

// Solid nodes: mask [nz][ny][nx], nonzero = solid (before o3_init).
void o3_set_solid(void* h, const uint8_t* mask) {
    Sim* s = static_cast<Sim*>(h);
    for (size_t n = 0; n < s->N; ++n) s->solid[n] = mask[n] ? 1 : 0;
}

// Relaxation times from the transport coefficients (Sec. 3.1-3.2), rho0 = 1.
int o3_set_params(void* h, double nu_s, double eta_p, double lam, double kappa, double Lambda_s,
                  double Lambda_p, double Fx, double Fy, double Fz, int no_source) {
    if (!(nu_s > 0) || !(kappa > 0) || !(lam > 0) || !(eta_p >= 0)) return -1;
    Sim* s = static_cast<Sim*>(h);
    s->p.tau_s1 = nu_s / CS2 + 0.5;
    s->p.tau_s2 = Lambda_s / (s->p.tau_s1 - 0.5) + 0.5;
    s->p.tau_p1 = kappa / CS2 + 0.5;
    s->p.tau_p2 = Lambda_p / (s->p.tau_p1 - 0.5) + 0.5;
    s->p.lam = lam;
    s->p.eta_p = eta_p;
    s->p.F[0] = Fx;
    s->p.F[1] = Fy;
    s->p.F[2] = Fz;
    s->p.no_source = no_source;
    return 0;
}

void o3_init(void* h, const double* rho, const double* ux, const double* uy, const double* uz,
             const double* a0, const double* a1, const double* a2, const double* a3,
             const double* a4, const double* a5) {
    const double* u[3] = {ux, uy, uz};
    const double* a[6] = {a0, a1, a2, a3, a4, a5};
    static_cast<Sim*>(h)->init(rho, u, a);
}

void o3_step(void* h, long long n) {
    Sim* s = static_cast<Sim*>(h);
    for (long long k = 0; k < n; ++k) s->step_once();
}

// rho, u (with the half-force shift) and the six conformation components.
void o3_read(void* h, double* rho, double* ux, double* uy, double* uz, double* a0, double* a1,
             double* a2, double* a3, double* a4, double* a5) {
    Sim* s = static_cast<Sim*>(h);
    s->macros();
    double* u[3] = {ux, uy, uz};
    double* a[6] = {a0, a1, a2, a3, a4, a5};
    for (size_t n = 0; n < s->N; ++n) {
        rho[n] = s->rho[n];
        for (int k = 0; k < 3; ++k) u[k][n] = s->u[k][n];
        for (int k = 0; k < 6; ++k) a[k][n] = s->A[k][n];
    }
}

// Lattice tables of D3Q19 or D3Q27 (q) and the third-order basis at every velocity
// (q x nb3, nb3 returned: 6 on D3Q19 -- h_{c,+}, h_{c,-} for c = 0, 1, 2 --, 7 on D3Q27 --
// H_xxy, H_xxz, H_yyx, H_yyz, H_zzx, H_zzy, H_xyz).  Arrays sized for 27 velocities and
// 7 basis functions.  Returns -1 for another q.
int o3_lattice(int q, int* e, double* w, int* opp, double* h3) {
    if (q != 19 && q != 27) return -1;
    const Lattice& L = q == 27 ? LAT27 : LAT19;
    for (int i = 0; i < L.Q; ++i) {
        for (int a = 0; a < 3; ++a) e[3 * i + a] = L.E[i][a];
        w[i] = L.W[i];
        opp[i] = L.OPP[i];
        for (int m = 0; m < L.nb3; ++m) h3[L.nb3 * i + m] = L.h3(i, m);
    }
    return L.nb3;
}

// One hydrodynamic collision at a single node (the collision of the step, exposed for
// the per-node pins): populations f (q values), rho, u, force F, polymer stress tau
// (row-major 3 x 3), the diagonal defects D, relaxation times tau_s1, tau_s2; out gets
// the q post-collision populations.  Returns -1 for another q.
int o3_collide_hydro(int q, const double* f, double rho, const double* u, const double* F,
                     const double* tau, const double* D, double tau_s1, double tau_s2,
                     double* out) {
    if (q != 19 && q != 27) return -1;
    Params p;
    p.tau_s1 = tau_s1;
    p.tau_s2 = tau_s2;
    double t[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) t[a][b] = tau[3 * a + b];
    collide_hydro(q == 27 ? LAT27 : LAT19, f, rho, u, F, t, D, p, out);
    return 0;
}

// One convection-diffusion collision at a single node: populations g (q values), phi,
// rho, u, force F, source S and its previous value Sp, previous velocity up, relaxation
// times tau_p1, tau_p2; out gets the q post-collision populations.  Returns -1 for
// another q.
int o3_collide_cde(int q, const double* g, double phi, double rho, const double* u,
                   const double* F, double S, double Sp, const double* up, double tau_p1,
                   double tau_p2, double* out) {
    if (q != 19 && q != 27) return -1;
    Params p;
    p.tau_p1 = tau_p1;
    p.tau_p2 = tau_p2;
    collide_cde(q == 27 ? LAT27 : LAT19, g, phi, rho, u, F, S, Sp, up, p, out);
    return 0;
}

// Constitutive closure (MODEL_*) and its parameter: Giesekus alpha in [0, 1], PTT eps >= 0,
// FENE-P L^2 > 3.  Returns -1 for an invalid pair.
int o3_set_model(void* h, int model, double mpar) {
    if (model < MODEL_OLDROYD_B || model > MODEL_FENE_P) return -1;
    if (model == MODEL_GIESEKUS && !(mpar >= 0.0 && mpar <= 1.0)) return -1;
    if ((model == MODEL_LPTT || model == MODEL_EPTT) && !(mpar >= 0.0)) return -1;
    if (model == MODEL_FENE_P && !(mpar > 3.0)) return -1;
    Sim* s = static_cast<Sim*>(h);
    s->p.model = model;
    s->p.mpar = model == MODEL_OLDROYD_B ? 0.0 : mpar;
    return 0;
}

// The constitutive source of a closure for a conformation A and velocity gradient
// L_gb = d_g u_b (both row-major 3 x 3), relaxation time lam, into S (row-major 3 x 3).
void o3_source_model(const double* A, const double* L, double lam, int model, double mpar,
                     double* S) {
    double a[3][3], l[3][3], s[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            a[i][j] = A[3 * i + j];
            l[i][j] = L[3 * i + j];
        }
    source3(a, l, lam, s, model, mpar);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) S[3 * i + j] = s[i][j];
}

// The constitutive source for a conformation A and velocity gradient L_gb = d_g u_b
// (both row-major 3 x 3), relaxation time lam, into S (row-major 3 x 3).
void o3_source(const double* A, const double* L, double lam, double* S) {
    double a[3][3], l[3][3], s[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            a[i][j] = A[3 * i + j];
            l[i][j] = L[3 * i + j];
        }
    source3(a, l, lam, s);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) S[3 * i + j] = s[i][j];
}

}  // extern "C"
