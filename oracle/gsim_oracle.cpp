/*
 * FP64 CPU oracle for the differentiable simulation step of "gradSim:
 * differentiable simulation for system identification and visuomotor control"
 * (ICLR 2021).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header,
 * table or helper with the HIP path under paper_2104_02646_amd/, and it
 * recomputes every rest quantity itself from the rest positions.
 *
 * What it computes, in the paper's order:
 *   - forces f(s) on particles from
 *       stable Neo-Hookean constant-strain tetrahedra (App. A.1 "Deformable
 *       Solids"; App. B.1, energy density Psi with Lame parameters and a
 *       per-element actuation alpha),
 *       Neo-Hookean constant-strain triangles embedded in 3D plus dihedral
 *       bending f_b = k_b sin(phi/2 + alpha) d with Bridson's direction d
 *       (App. A.1 "Deformable Thin-Shells"),
 *       compliant ground contact f_n = -n[k_e C + k_d Cdot] and relaxed
 *       Coulomb friction -D[min(mu |f_n|, k_f u_s)] against a plane
 *       (App. A.1 "Contact", App. B.2);
 *   - the semi-implicit Euler step u+ = u- + dt M^-1 f(s-), q+ = q- + dt u+
 *       (App. A.2 residual g(s-, s+, theta) = 0, App. C integration kernel);
 *   - a rollout of T steps and the mean-squared position loss;
 *   - the discrete adjoint of that rollout (App. A, implicit-function
 *       theorem; App. A.2 step Jacobians, whose block-triangular structure
 *       makes each reverse step explicit).  The element Jacobians used in the
 *       reverse step are obtained by forward-mode dual numbers in FP64, so the
 *       adjoint shares no hand derivation with the GPU path.
 *
 * Readings where the paper is silent (recorded with the design notes):
 *   R1  alpha = 1 + 3 mu / (4 lambda) + a_e (rest-stable, a_e = actuation);
 *   R2  membrane: 2D stable Neo-Hookean, mu = lambda = k_t,
 *       alpha2 = 1 + 2 mu / (3 lambda), energy mu/2(Ic-2) + lambda/2(J-alpha2)^2
 *       - mu/2 log(Ic+1);
 *   R3  bending scale |E|^2 / (|N1| + |N2|), rest angle phi0 from the rest mesh;
 *   R4  f_n = +lambda_n n with n the outward plane normal;
 *   R5  contact when n.x - d < 0 (threshold 0);
 *   R6  isotropic friction cone, stick when k_f |u_t| <= mu_f |lambda_n|;
 *   R8  all forces evaluated at the step-start state;
 *   R9  gravity acceleration applied to free particles only (w > 0).
 *
 * Build: g++ -O2 -ffp-contract=off -fno-fast-math (no FMA contraction).
 * Layout: every array is AoS [n][3] double unless stated.
 */
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

namespace {

/* ---------------------------------------------------------------------- */
/* Forward-mode dual numbers: value plus ND tangent components.            */
/* ---------------------------------------------------------------------- */
const int ND = 16;

struct Dual {
    double v;
    double d[ND];
    Dual() : v(0.0) { for (int k = 0; k < ND; ++k) d[k] = 0.0; }
    Dual(double x) : v(x) { for (int k = 0; k < ND; ++k) d[k] = 0.0; }
};

Dual operator+(const Dual& a, const Dual& b) { Dual r(a.v + b.v); for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] + b.d[k]; return r; }
Dual operator-(const Dual& a, const Dual& b) { Dual r(a.v - b.v); for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] - b.d[k]; return r; }
Dual operator-(const Dual& a) { Dual r(-a.v); for (int k = 0; k < ND; ++k) r.d[k] = -a.d[k]; return r; }
Dual operator*(const Dual& a, const Dual& b) { Dual r(a.v * b.v); for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k]; return r; }
Dual operator/(const Dual& a, const Dual& b) {
    Dual r(a.v / b.v);
    for (int k = 0; k < ND; ++k) r.d[k] = (a.d[k] * b.v - a.v * b.d[k]) / (b.v * b.v);
    return r;
}
Dual operator+(const Dual& a, double b) { return a + Dual(b); }
Dual operator+(double a, const Dual& b) { return Dual(a) + b; }
Dual operator-(const Dual& a, double b) { return a - Dual(b); }
Dual operator-(double a, const Dual& b) { return Dual(a) - b; }
Dual operator*(const Dual& a, double b) { return a * Dual(b); }
Dual operator*(double a, const Dual& b) { return Dual(a) * b; }
Dual operator/(const Dual& a, double b) { return a / Dual(b); }
Dual operator/(double a, const Dual& b) { return Dual(a) / b; }

Dual sqrt(const Dual& a) {
    Dual r(std::sqrt(a.v));
    for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] / (2.0 * r.v);
    return r;
}
Dual log(const Dual& a) { Dual r(std::log(a.v)); for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] / a.v; return r; }
Dual sin(const Dual& a) { Dual r(std::sin(a.v)); double c = std::cos(a.v); for (int k = 0; k < ND; ++k) r.d[k] = c * a.d[k]; return r; }
Dual atan2(const Dual& y, const Dual& x) {
    Dual r(std::atan2(y.v, x.v));
    double q = x.v * x.v + y.v * y.v;
    for (int k = 0; k < ND; ++k) r.d[k] = (x.v * y.d[k] - y.v * x.d[k]) / q;
    return r;
}
Dual fabs(const Dual& a) { return a.v < 0.0 ? -a : a; }

/* The same names for plain doubles, so the templates below read alike for
 * both scalar types. */
double sqrt(double a) { return std::sqrt(a); }
double log(double a) { return std::log(a); }
double sin(double a) { return std::sin(a); }
double atan2(double y, double x) { return std::atan2(y, x); }
double fabs(double a) { return std::fabs(a); }

double val(double a) { return a; }
double val(const Dual& a) { return a.v; }

/* ---------------------------------------------------------------------- */
/* 3-vectors over a scalar type S (double or Dual).                        */
/* ---------------------------------------------------------------------- */
template <class S> struct V3 { S x, y, z; };
template <class S> struct Same { typedef S type; }; /* blocks deduction from the scalar argument */

template <class S> V3<S> mk(S x, S y, S z) { V3<S> r; r.x = x; r.y = y; r.z = z; return r; }
template <class S> V3<S> operator+(const V3<S>& a, const V3<S>& b) { return mk<S>(a.x + b.x, a.y + b.y, a.z + b.z); }
template <class S> V3<S> operator-(const V3<S>& a, const V3<S>& b) { return mk<S>(a.x - b.x, a.y - b.y, a.z - b.z); }
template <class S> V3<S> operator-(const V3<S>& a) { return mk<S>(-a.x, -a.y, -a.z); }
template <class S> V3<S> operator*(const V3<S>& a, const typename Same<S>::type& s) { return mk<S>(a.x * s, a.y * s, a.z * s); }
template <class S> S dot(const V3<S>& a, const V3<S>& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class S> V3<S> cross(const V3<S>& a, const V3<S>& b) {
    return mk<S>(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
template <class S> S norm(const V3<S>& a) { return sqrt(dot(a, a)); }
template <class S> V3<S> zero3() { return mk<S>(S(0.0), S(0.0), S(0.0)); }

V3<double> load3(const double* p) { return mk<double>(p[0], p[1], p[2]); }
void store3(double* p, const V3<double>& a) { p[0] = a.x; p[1] = a.y; p[2] = a.z; }
void add3(double* p, const V3<double>& a) { p[0] += a.x; p[1] += a.y; p[2] += a.z; }

/* ---------------------------------------------------------------------- */
/* Rest-state quantities (recomputed here from the rest positions).        */
/* ---------------------------------------------------------------------- */

/* Dm = [X1-X0, X2-X0, X3-X0] (columns); DmInv row-major 3x3; V = det(Dm)/6. */
double tet_rest(const V3<double> X[4], double DmInv[9]) {
    V3<double> c0 = X[1] - X[0], c1 = X[2] - X[0], c2 = X[3] - X[0];
    double Dm[3][3] = {{c0.x, c1.x, c2.x}, {c0.y, c1.y, c2.y}, {c0.z, c1.z, c2.z}};
    double det = Dm[0][0] * (Dm[1][1] * Dm[2][2] - Dm[1][2] * Dm[2][1])
               - Dm[0][1] * (Dm[1][0] * Dm[2][2] - Dm[1][2] * Dm[2][0])
               + Dm[0][2] * (Dm[1][0] * Dm[2][1] - Dm[1][1] * Dm[2][0]);
    /* inverse = adjugate / det */
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            int r1 = (c + 1) % 3, r2 = (c + 2) % 3, c1i = (r + 1) % 3, c2i = (r + 2) % 3;
            DmInv[r * 3 + c] = (Dm[r1][c1i] * Dm[r2][c2i] - Dm[r1][c2i] * Dm[r2][c1i]) / det;
        }
    return det;
}

/* In-plane rest frame e1 = (X1-X0)/|X1-X0|, e2 = n x e1 with n the unit
 * normal of (X1-X0)x(X2-X0); Dm is the 2x2 matrix of the edge vectors in that
 * frame; A = det(Dm)/2.  DmInv row-major 2x2. */
double tri_rest(const V3<double> X[3], double DmInv[4]) {
    V3<double> a = X[1] - X[0], b = X[2] - X[0];
    V3<double> nrm = cross(a, b);
    nrm = nrm * (1.0 / norm(nrm));
    V3<double> e1 = a * (1.0 / norm(a));
    V3<double> e2 = cross(nrm, e1);
    double m00 = dot(e1, a), m01 = dot(e1, b), m10 = dot(e2, a), m11 = dot(e2, b);
    double det = m00 * m11 - m01 * m10;
    DmInv[0] = m11 / det; DmInv[1] = -m01 / det; DmInv[2] = -m10 / det; DmInv[3] = m00 / det;
    return 0.5 * det;
}

/* ---------------------------------------------------------------------- */
/* Element models.                                                         */
/* ---------------------------------------------------------------------- */

/* Deformation gradient of a tet: F = Ds Dm^-1, Ds = [x1-x0, x2-x0, x3-x0]. */
template <class S> void tet_F(const V3<S> x[4], const double DmInv[9], V3<S> F[3]) {
    V3<S> d[3] = {x[1] - x[0], x[2] - x[0], x[3] - x[0]};
    for (int j = 0; j < 3; ++j)
        F[j] = d[0] * DmInv[0 * 3 + j] + d[1] * DmInv[1 * 3 + j] + d[2] * DmInv[2 * 3 + j];
}

/* Strain energy of one tet, V * Psi with
 * Psi = mu/2 (Ic - 3) + lambda/2 (J - alpha)^2 - mu/2 log(Ic + 1)
 * (App. A.1, App. B.1), alpha per reading R1. */
template <class S> S tet_energy(const V3<S> x[4], const double DmInv[9], double V, S mu, S lam, S act) {
    V3<S> F[3];
    tet_F(x, DmInv, F);
    S Ic = dot(F[0], F[0]) + dot(F[1], F[1]) + dot(F[2], F[2]);
    S J = dot(F[0], cross(F[1], F[2]));
    S alpha = 1.0 + 0.75 * mu / lam + act;
    S psi = 0.5 * mu * (Ic - 3.0) + 0.5 * lam * (J - alpha) * (J - alpha) - 0.5 * mu * log(Ic + 1.0);
    return psi * V;
}

/* Corner forces f = -dE/dx of one tet.  First Piola stress
 * P = dPsi/dF = mu (1 - 1/(Ic+1)) F + lambda (J - alpha) cof(F), where
 * cof(F) = dJ/dF has columns F1xF2, F2xF0, F0xF1.  Then
 * [f1 f2 f3] = -V P Dm^-T and f0 = -(f1+f2+f3). */
template <class S>
void tet_force(const V3<S> x[4], const double DmInv[9], double V, S mu, S lam, S act, V3<S> f[4]) {
    V3<S> F[3];
    tet_F(x, DmInv, F);
    S Ic = dot(F[0], F[0]) + dot(F[1], F[1]) + dot(F[2], F[2]);
    V3<S> C[3] = {cross(F[1], F[2]), cross(F[2], F[0]), cross(F[0], F[1])};
    S J = dot(F[0], C[0]);
    S alpha = 1.0 + 0.75 * mu / lam + act;
    S a = mu * (1.0 - 1.0 / (Ic + 1.0));
    S b = lam * (J - alpha);
    V3<S> P[3];
    for (int j = 0; j < 3; ++j) P[j] = F[j] * a + C[j] * b;
    f[0] = zero3<S>();
    for (int i = 0; i < 3; ++i) {
        V3<S> h = P[0] * DmInv[i * 3 + 0] + P[1] * DmInv[i * 3 + 1] + P[2] * DmInv[i * 3 + 2];
        f[i + 1] = h * (-V);
        f[0] = f[0] - f[i + 1];
    }
}

/* Membrane deformation gradient (3x2): F = [x1-x0, x2-x0] Dm^-1. */
template <class S> void tri_F(const V3<S> x[3], const double DmInv[4], V3<S> F[2]) {
    V3<S> d1 = x[1] - x[0], d2 = x[2] - x[0];
    F[0] = d1 * DmInv[0] + d2 * DmInv[2];
    F[1] = d1 * DmInv[1] + d2 * DmInv[3];
}

/* Membrane energy A * Psi2 (reading R2): mu = lambda = k,
 * Psi2 = mu/2 (Ic - 2) + lambda/2 (J - alpha2)^2 - mu/2 log(Ic + 1),
 * J = |F0 x F1| (area ratio), alpha2 = 1 + 2 mu / (3 lambda). */
template <class S> S tri_energy(const V3<S> x[3], const double DmInv[4], double A, S k) {
    V3<S> F[2];
    tri_F(x, DmInv, F);
    S mu = k, lam = k;
    S Ic = dot(F[0], F[0]) + dot(F[1], F[1]);
    S J = norm(cross(F[0], F[1]));
    S alpha = 1.0 + (2.0 / 3.0) * mu / lam;
    S psi = 0.5 * mu * (Ic - 2.0) + 0.5 * lam * (J - alpha) * (J - alpha) - 0.5 * mu * log(Ic + 1.0);
    return psi * A;
}

/* Membrane corner forces: P = mu (1 - 1/(Ic+1)) F + lambda (J - alpha2) dJ/dF with
 * dJ/dF = [F1 x n, n x F0], n = (F0 x F1)/J; [f1 f2] = -A P Dm^-T, f0 = -(f1+f2). */
template <class S> void tri_force(const V3<S> x[3], const double DmInv[4], double A, S k, V3<S> f[3]) {
    V3<S> F[2];
    tri_F(x, DmInv, F);
    S mu = k, lam = k;
    S Ic = dot(F[0], F[0]) + dot(F[1], F[1]);
    V3<S> c = cross(F[0], F[1]);
    S J = norm(c);
    V3<S> n = c * (1.0 / J);
    V3<S> dJ[2] = {cross(F[1], n), cross(n, F[0])};
    S alpha = 1.0 + (2.0 / 3.0) * mu / lam;
    S a = mu * (1.0 - 1.0 / (Ic + 1.0));
    S b = lam * (J - alpha);
    V3<S> P[2] = {F[0] * a + dJ[0] * b, F[1] * a + dJ[1] * b};
    f[1] = (P[0] * DmInv[0] + P[1] * DmInv[1]) * (-A);
    f[2] = (P[0] * DmInv[2] + P[1] * DmInv[3]) * (-A);
    f[0] = -(f[1] + f[2]);
}

/* Signed dihedral angle of a hinge: x0, x1 are the wing vertices, x2 -> x3
 * the shared edge E.  N1 = (x0-x2)x(x0-x3), N2 = (x1-x3)x(x1-x2);
 * phi = atan2(-(n1 x n2).E/|E|, n1.n2).  The sign makes Bridson's u_i
 * (below) the exact gradient d phi / d x_i. */
template <class S> S hinge_angle(const V3<S> x[4]) {
    V3<S> E = x[3] - x[2];
    V3<S> N1 = cross(x[0] - x[2], x[0] - x[3]);
    V3<S> N2 = cross(x[1] - x[3], x[1] - x[2]);
    V3<S> n1 = N1 * (1.0 / norm(N1));
    V3<S> n2 = N2 * (1.0 / norm(N2));
    S sinp = dot(cross(n1, n2), E) / norm(E);
    S cosp = dot(n1, n2);
    return atan2(-sinp, cosp);
}

/* Bending force of one hinge (App. A.1 thin shells): f_i = -k_b s sin((phi-phi0)/2 + alpha) u_i
 * with s = |E|^2 / (|N1| + |N2|) and Bridson's directions
 *   u0 = |E| N1/|N1|^2, u1 = |E| N2/|N2|^2,
 *   u2 = ((x0-x3).E/|E|) N1/|N1|^2 + ((x1-x3).E/|E|) N2/|N2|^2,
 *   u3 = -((x0-x2).E/|E|) N1/|N1|^2 - ((x1-x2).E/|E|) N2/|N2|^2.
 * The minus sign makes the force restoring (reading R3). */
template <class S> void hinge_force(const V3<S> x[4], double phi0, S kb, S act, V3<S> f[4]) {
    V3<S> E = x[3] - x[2];
    V3<S> N1 = cross(x[0] - x[2], x[0] - x[3]);
    V3<S> N2 = cross(x[1] - x[3], x[1] - x[2]);
    S el = norm(E);
    S n1sq = dot(N1, N1), n2sq = dot(N2, N2);
    V3<S> a1 = N1 * (1.0 / n1sq), a2 = N2 * (1.0 / n2sq);
    V3<S> u[4];
    u[0] = a1 * el;
    u[1] = a2 * el;
    u[2] = a1 * (dot(x[0] - x[3], E) / el) + a2 * (dot(x[1] - x[3], E) / el);
    u[3] = -(a1 * (dot(x[0] - x[2], E) / el) + a2 * (dot(x[1] - x[2], E) / el));
    S phi = hinge_angle(x);
    S s = el * el / (sqrt(n1sq) + sqrt(n2sq));
    S mag = -(kb * s * sin(0.5 * (phi - phi0) + act));
    for (int i = 0; i < 4; ++i) f[i] = u[i] * mag;
}

/* Ground contact on one particle (App. A.1 "Contact", App. B.2, readings R4-R6):
 * gap = n.x - d, C = max(0, -gap); when C > 0,
 * lambda_n = k_e C + k_d Cdot with Cdot = -n.v, f_n = lambda_n n,
 * u_t = v - (n.v) n, stick (k_f |u_t| <= mu_f |lambda_n|): f_f = -k_f u_t,
 * slip: f_f = -mu_f |lambda_n| u_t / |u_t|. */
template <class S>
V3<S> contact_force(const V3<S>& x, const V3<S>& v, const double nrm[4], S ke, S kd, S kf, S muf) {
    V3<S> n = mk<S>(S(nrm[0]), S(nrm[1]), S(nrm[2]));
    S gap = dot(n, x) - nrm[3];
    if (!(val(gap) < 0.0)) return zero3<S>();
    S C = -gap;
    S Cdot = -dot(n, v);
    S lam_n = ke * C + kd * Cdot;
    V3<S> fn = n * lam_n;
    V3<S> ut = v - n * dot(n, v);
    double sval = std::sqrt(val(dot(ut, ut)));
    S limit = muf * fabs(lam_n);
    V3<S> ff;
    if (val(kf) * sval <= val(limit)) {
        ff = ut * (-kf);
    } else {
        S s = norm(ut);
        ff = ut * (-(limit / s));
    }
    return fn + ff;
}

/* Air force on one cloth triangle (App. A.1 thin shells: a lift/drag model of the
 * surrounding air; the paper gives no formula, reading R20).  Still air; u is the
 * mean corner velocity, n the unit normal, A the current area, s = n.u:
 *   drag  F_d = -k_d A |s| u                          (quadratic, projected area)
 *   lift  F_l = -k_l A s (|u|^2 n - s u) / |u|          (flat plate: perpendicular
 *         to u, magnitude k_l A |u|^2 sin(2 a) / 2 for the angle a between u and
 *         the plate; F_l = 0 at u = 0, where it and its Jacobian vanish)
 * and each corner receives (F_d + F_l) / 3. */
template <class S>
void air_force(const V3<S> x[3], const V3<S> v[3], S kd, S kl, V3<S> f[3]) {
    V3<S> N = cross(x[1] - x[0], x[2] - x[0]);
    S nn = norm(N);
    V3<S> n = N * (1.0 / nn);
    S A = 0.5 * nn;
    V3<S> u = (v[0] + v[1] + v[2]) * (1.0 / 3.0);
    S s = dot(n, u);
    S q = dot(u, u);
    V3<S> F = u * (-(kd * A * fabs(s)));
    if (val(q) > 0.0) {
        S r = sqrt(q);
        F = F + (n * q - u * s) * (-(kl * A * s / r));
    }
    for (int i = 0; i < 3; ++i) f[i] = F * (1.0 / 3.0);
}

/* One-sided quadratic contact potential k_e C^2 / 2 (its negative gradient is
 * the elastic part of f_n). */
double contact_energy(const V3<double>& x, const double nrm[4], double ke) {
    double gap = nrm[0] * x.x + nrm[1] * x.y + nrm[2] * x.z - nrm[3];
    if (!(gap < 0.0)) return 0.0;
    return 0.5 * ke * gap * gap;
}

/* ---------------------------------------------------------------------- */
/* Model: topology, rest data, environment.                                */
/* ---------------------------------------------------------------------- */
struct Model {
    int np, ne, nt, nh;
    std::vector<double> X;
    std::vector<int> tet, tri, hinge;
    std::vector<double> tetDmInv, tetV, triDmInv, triA, phi0;
    std::vector<unsigned char> pinned;
    double g[3];
    int ground;
    int air;  /* lift/drag on the triangles */
    double plane[4];
    double dt;
    int status;
};

}  // namespace

extern "C" {

typedef struct {
    const double *mu, *lam, *act; /* [ne]; act may be NULL (zero) */
    const double *ktri;           /* [nt] */
    const double *hact;           /* [nh] or NULL (zero) */
    const double *mass;           /* [np] */
    double kb;                    /* bending stiffness (per body) */
    double ke, kd, kf, muf;       /* contact parameters */
    double kdrag, klift;          /* air force coefficients (used when the model has air on) */
} oc_params;

typedef struct {
    double *mu, *lam, *act, *ktri, *hact, *mass; /* NULL = not requested */
    double kb;
    double contact[4]; /* ke, kd, kf, muf */
    double air[2];     /* kdrag, klift */
} oc_grads;

}  // extern "C"

namespace {

double act_of(const oc_params* p, int e) { return p->act ? p->act[e] : 0.0; }
double hact_of(const oc_params* p, int h) { return p->hact ? p->hact[h] : 0.0; }
double inv_mass(const Model* m, const oc_params* p, int i) { return m->pinned[i] ? 0.0 : 1.0 / p->mass[i]; }

/* Total force f(x, v) = sum of element forces + contact (sequential scatter). */
void total_force(const Model* m, const oc_params* p, const double* x, const double* v, double* f) {
    std::memset(f, 0, sizeof(double) * 3 * m->np);
    for (int e = 0; e < m->ne; ++e) {
        const int* id = &m->tet[4 * e];
        V3<double> xe[4], fe[4];
        for (int k = 0; k < 4; ++k) xe[k] = load3(&x[3 * id[k]]);
        tet_force<double>(xe, &m->tetDmInv[9 * e], m->tetV[e], p->mu[e], p->lam[e], act_of(p, e), fe);
        for (int k = 0; k < 4; ++k) add3(&f[3 * id[k]], fe[k]);
    }
    for (int t = 0; t < m->nt; ++t) {
        const int* id = &m->tri[3 * t];
        V3<double> xe[3], fe[3];
        for (int k = 0; k < 3; ++k) xe[k] = load3(&x[3 * id[k]]);
        tri_force<double>(xe, &m->triDmInv[4 * t], m->triA[t], p->ktri[t], fe);
        for (int k = 0; k < 3; ++k) add3(&f[3 * id[k]], fe[k]);
        if (m->air) {
            V3<double> ve[3];
            for (int k = 0; k < 3; ++k) ve[k] = load3(&v[3 * id[k]]);
            air_force<double>(xe, ve, p->kdrag, p->klift, fe);
            for (int k = 0; k < 3; ++k) add3(&f[3 * id[k]], fe[k]);
        }
    }
    for (int h = 0; h < m->nh; ++h) {
        const int* id = &m->hinge[4 * h];
        V3<double> xe[4], fe[4];
        for (int k = 0; k < 4; ++k) xe[k] = load3(&x[3 * id[k]]);
        hinge_force<double>(xe, m->phi0[h], p->kb, hact_of(p, h), fe);
        for (int k = 0; k < 4; ++k) add3(&f[3 * id[k]], fe[k]);
    }
    if (m->ground) {
        for (int i = 0; i < m->np; ++i) {
            V3<double> fc = contact_force<double>(load3(&x[3 * i]), load3(&v[3 * i]), m->plane, p->ke, p->kd, p->kf, p->muf);
            add3(&f[3 * i], fc);
        }
    }
}

/* Semi-implicit Euler (App. A.2): v+ = v + dt (w f + g [w > 0]), x+ = x + dt v+. */
void step(const Model* m, const oc_params* p, const double* x, const double* v, double* xo, double* vo,
          std::vector<double>& f) {
    total_force(m, p, x, v, f.data());
    for (int i = 0; i < m->np; ++i) {
        double w = inv_mass(m, p, i);
        double gate = w > 0.0 ? 1.0 : 0.0;
        for (int c = 0; c < 3; ++c) {
            double vn = v[3 * i + c] + m->dt * (w * f[3 * i + c] + m->g[c] * gate);
            vo[3 * i + c] = vn;
            xo[3 * i + c] = x[3 * i + c] + m->dt * vn;
        }
    }
}

/* Seed dual tangents: component k of corner c gets tangent slot 3c+k. */
template <int NC> void seed_positions(const double* x, const int* id, V3<Dual> xe[NC]) {
    for (int c = 0; c < NC; ++c) {
        const double* p = &x[3 * id[c]];
        xe[c] = mk<Dual>(Dual(p[0]), Dual(p[1]), Dual(p[2]));
        xe[c].x.d[3 * c + 0] = 1.0;
        xe[c].y.d[3 * c + 1] = 1.0;
        xe[c].z.d[3 * c + 2] = 1.0;
    }
}

Dual dvar(double v, int slot) { Dual r(v); r.d[slot] = 1.0; return r; }

/* Apply the transpose of an element's force Jacobian to the adjoint force:
 * xbar[id[c]] += sum_i (d f_i / d x_c)^T fbar[id[i]], with the Jacobian read
 * from the dual tangents (slot 3c+k is d/d x_c[k]).  Returns, in pbar[s],
 * sum_i fbar_i . d f_i / d(tangent slot s) for the parameter slots. */
template <int NC>
void apply_transpose(const V3<Dual> fe[NC], const int* id, const double* fbar, double* xbar, double* pbar_slots) {
    for (int s = 0; s < ND; ++s) {
        double acc = 0.0;
        for (int i = 0; i < NC; ++i) {
            const double* fb = &fbar[3 * id[i]];
            acc += fb[0] * fe[i].x.d[s] + fb[1] * fe[i].y.d[s] + fb[2] * fe[i].z.d[s];
        }
        if (s < 3 * NC)
            xbar[3 * id[s / 3] + (s % 3)] += acc;
        else
            pbar_slots[s] = acc;
    }
}

/* Adjoint of the total force: given fbar, accumulate (df/dx)^T fbar into xbar,
 * (df/dv)^T fbar into vbar, and (df/dtheta)^T fbar into the parameter grads. */
void force_vjp(const Model* m, const oc_params* p, const double* x, const double* v, const double* fbar, double* xbar,
               double* vbar, oc_grads* g) {
    double pb[ND];
    for (int e = 0; e < m->ne; ++e) {
        const int* id = &m->tet[4 * e];
        V3<Dual> xe[4], fe[4];
        seed_positions<4>(x, id, xe);
        Dual mu = dvar(p->mu[e], 12), lam = dvar(p->lam[e], 13), act = dvar(act_of(p, e), 14);
        tet_force<Dual>(xe, &m->tetDmInv[9 * e], m->tetV[e], mu, lam, act, fe);
        for (int s = 0; s < ND; ++s) pb[s] = 0.0;
        apply_transpose<4>(fe, id, fbar, xbar, pb);
        if (g) {
            if (g->mu) g->mu[e] += pb[12];
            if (g->lam) g->lam[e] += pb[13];
            if (g->act) g->act[e] += pb[14];
        }
    }
    for (int t = 0; t < m->nt; ++t) {
        const int* id = &m->tri[3 * t];
        V3<Dual> xe[3], fe[3];
        seed_positions<3>(x, id, xe);
        Dual k = dvar(p->ktri[t], 9);
        tri_force<Dual>(xe, &m->triDmInv[4 * t], m->triA[t], k, fe);
        for (int s = 0; s < ND; ++s) pb[s] = 0.0;
        apply_transpose<3>(fe, id, fbar, xbar, pb);
        if (g && g->ktri) g->ktri[t] += pb[9];
        if (m->air) {
            /* two passes: positions and the coefficients, then velocities */
            V3<Dual> ve[3];
            for (int c = 0; c < 3; ++c) ve[c] = mk<Dual>(Dual(v[3 * id[c]]), Dual(v[3 * id[c] + 1]), Dual(v[3 * id[c] + 2]));
            air_force<Dual>(xe, ve, dvar(p->kdrag, 9), dvar(p->klift, 10), fe);
            for (int s = 0; s < ND; ++s) pb[s] = 0.0;
            apply_transpose<3>(fe, id, fbar, xbar, pb);
            if (g) {
                g->air[0] += pb[9];
                g->air[1] += pb[10];
            }
            for (int c = 0; c < 3; ++c) xe[c] = mk<Dual>(Dual(x[3 * id[c]]), Dual(x[3 * id[c] + 1]), Dual(x[3 * id[c] + 2]));
            seed_positions<3>(v, id, ve);
            air_force<Dual>(xe, ve, Dual(p->kdrag), Dual(p->klift), fe);
            apply_transpose<3>(fe, id, fbar, vbar, pb);
        }
    }
    for (int h = 0; h < m->nh; ++h) {
        const int* id = &m->hinge[4 * h];
        V3<Dual> xe[4], fe[4];
        seed_positions<4>(x, id, xe);
        Dual kb = dvar(p->kb, 12), ha = dvar(hact_of(p, h), 13);
        hinge_force<Dual>(xe, m->phi0[h], kb, ha, fe);
        for (int s = 0; s < ND; ++s) pb[s] = 0.0;
        apply_transpose<4>(fe, id, fbar, xbar, pb);
        if (g) {
            g->kb += pb[12];
            if (g->hact) g->hact[h] += pb[13];
        }
    }
    if (m->ground) {
        for (int i = 0; i < m->np; ++i) {
            const double* xi = &x[3 * i];
            const double* vi = &v[3 * i];
            V3<Dual> xd = mk<Dual>(dvar(xi[0], 0), dvar(xi[1], 1), dvar(xi[2], 2));
            V3<Dual> vd = mk<Dual>(dvar(vi[0], 3), dvar(vi[1], 4), dvar(vi[2], 5));
            Dual ke = dvar(p->ke, 6), kd = dvar(p->kd, 7), kf = dvar(p->kf, 8), muf = dvar(p->muf, 9);
            V3<Dual> fc = contact_force<Dual>(xd, vd, m->plane, ke, kd, kf, muf);
            const double* fb = &fbar[3 * i];
            double acc[10];
            for (int s = 0; s < 10; ++s) acc[s] = fb[0] * fc.x.d[s] + fb[1] * fc.y.d[s] + fb[2] * fc.z.d[s];
            for (int k = 0; k < 3; ++k) {
                xbar[3 * i + k] += acc[k];
                vbar[3 * i + k] += acc[3 + k];
            }
            if (g)
                for (int k = 0; k < 4; ++k) g->contact[k] += acc[6 + k];
        }
    }
}

/* One reverse step of semi-implicit Euler (App. A.2 Jacobians).
 * Forward: v+ = v + dt (w f(x, v) + g [w>0]), x+ = x + dt v+.
 * Given (xbar+, vbar+): vt = vbar+ + dt xbar+ is the total adjoint of v+;
 * fbar = dt w vt; wbar = dt f . vt; xbar- = xbar+ + (df/dx)^T fbar;
 * vbar- = vt + (df/dv)^T fbar; theta-bar += (df/dtheta)^T fbar;
 * mass: w = 1/m so mbar = -w^2 wbar (free particles only). */
void step_vjp(const Model* m, const oc_params* p, const double* x, const double* v, const double* xbp,
              const double* vbp, double* xbm, double* vbm, oc_grads* g, std::vector<double>& f,
              std::vector<double>& fbar) {
    total_force(m, p, x, v, f.data());
    for (int i = 0; i < m->np; ++i) {
        double w = inv_mass(m, p, i);
        double wbar = 0.0;
        for (int c = 0; c < 3; ++c) {
            double vt = vbp[3 * i + c] + m->dt * xbp[3 * i + c];
            fbar[3 * i + c] = m->dt * w * vt;
            wbar += m->dt * f[3 * i + c] * vt;
            xbm[3 * i + c] = xbp[3 * i + c];
            vbm[3 * i + c] = vt;
        }
        if (g && g->mass && w > 0.0) g->mass[i] += -w * w * wbar;
    }
    force_vjp(m, p, x, v, fbar.data(), xbm, vbm, g);
}

}  // namespace

extern "C" {

/* Creates an oracle model.  X [np][3] rest positions; tet [ne][4];
 * tri [nt][3]; hinge [nh][4] (wing0, wing1, edge0, edge1); pinned [np];
 * gravity [3]; plane [4] = (n, d) with unit n; ground != 0 enables contact.
 * Negatively oriented tets are reordered (swap of corners 1 and 2).
 * Status (oc_status): 0 ok, -2 index out of range, -3 degenerate element. */
void* oc_create(int np, int ne, int nt, int nh, const double* X, const int* tet, const int* tri, const int* hinge,
                const unsigned char* pinned, const double* gravity, int ground, const double* plane, double dt) {
    Model* m = new Model();
    m->np = np; m->ne = ne; m->nt = nt; m->nh = nh;
    m->X.assign(X, X + 3 * (size_t)np);
    m->tet.assign(tet, tet + 4 * (size_t)ne);
    m->tri.assign(tri, tri + 3 * (size_t)nt);
    m->hinge.assign(hinge, hinge + 4 * (size_t)nh);
    m->pinned.assign(np, 0);
    if (pinned) for (int i = 0; i < np; ++i) m->pinned[i] = pinned[i] ? 1 : 0;
    for (int c = 0; c < 3; ++c) m->g[c] = gravity[c];
    m->ground = ground;
    m->air = 0;
    for (int c = 0; c < 4; ++c) m->plane[c] = plane ? plane[c] : (c == 1 ? 1.0 : 0.0);
    m->dt = dt;
    m->status = 0;
    for (size_t k = 0; k < m->tet.size(); ++k) if (m->tet[k] < 0 || m->tet[k] >= np) m->status = -2;
    for (size_t k = 0; k < m->tri.size(); ++k) if (m->tri[k] < 0 || m->tri[k] >= np) m->status = -2;
    for (size_t k = 0; k < m->hinge.size(); ++k) if (m->hinge[k] < 0 || m->hinge[k] >= np) m->status = -2;
    if (m->status) return m;
    m->tetDmInv.resize(9 * (size_t)ne); m->tetV.resize(ne);
    for (int e = 0; e < ne; ++e) {
        V3<double> Xe[4];
        for (int k = 0; k < 4; ++k) Xe[k] = load3(&X[3 * m->tet[4 * e + k]]);
        double det = tet_rest(Xe, &m->tetDmInv[9 * e]);
        if (det < 0.0) {
            int t = m->tet[4 * e + 1]; m->tet[4 * e + 1] = m->tet[4 * e + 2]; m->tet[4 * e + 2] = t;
            for (int k = 0; k < 4; ++k) Xe[k] = load3(&X[3 * m->tet[4 * e + k]]);
            det = tet_rest(Xe, &m->tetDmInv[9 * e]);
        }
        if (!(det > 0.0)) m->status = -3;
        m->tetV[e] = det / 6.0;
    }
    m->triDmInv.resize(4 * (size_t)nt); m->triA.resize(nt);
    for (int t = 0; t < nt; ++t) {
        V3<double> Xe[3];
        for (int k = 0; k < 3; ++k) Xe[k] = load3(&X[3 * m->tri[3 * t + k]]);
        m->triA[t] = tri_rest(Xe, &m->triDmInv[4 * t]);
        if (!(m->triA[t] > 0.0)) m->status = -3;
    }
    m->phi0.resize(nh);
    for (int h = 0; h < nh; ++h) {
        V3<double> Xe[4];
        for (int k = 0; k < 4; ++k) Xe[k] = load3(&X[3 * m->hinge[4 * h + k]]);
        m->phi0[h] = hinge_angle<double>(Xe);
    }
    return m;
}

int oc_status(void* h) { return static_cast<Model*>(h)->status; }
/* Switches the lift/drag force on the triangles on (nonzero) or off. */
void oc_set_air(void* h, int on) { static_cast<Model*>(h)->air = on ? 1 : 0; }
void oc_free(void* h) { delete static_cast<Model*>(h); }

/* Rest data as computed by the oracle (for inspection in tests). */
void oc_rest_data(void* h, double* tetV, double* triA, double* phi0) {
    Model* m = static_cast<Model*>(h);
    if (tetV) for (int e = 0; e < m->ne; ++e) tetV[e] = m->tetV[e];
    if (triA) for (int t = 0; t < m->nt; ++t) triA[t] = m->triA[t];
    if (phi0) for (int k = 0; k < m->nh; ++k) phi0[k] = m->phi0[k];
}

/* Total force f(x, v), AoS [np][3]. */
int oc_forces(void* h, const oc_params* p, const double* x, const double* v, double* f) {
    Model* m = static_cast<Model*>(h);
    if (m->status) return m->status;
    total_force(m, p, x, v, f);
    return 0;
}

/* Potential energy of the conservative forces: tet and membrane strain
 * energy plus the contact penalty potential (bending has no potential in
 * this model and is excluded). */
double oc_energy(void* h, const oc_params* p, const double* x) {
    Model* m = static_cast<Model*>(h);
    double E = 0.0;
    for (int e = 0; e < m->ne; ++e) {
        V3<double> xe[4];
        for (int k = 0; k < 4; ++k) xe[k] = load3(&x[3 * m->tet[4 * e + k]]);
        E += tet_energy<double>(xe, &m->tetDmInv[9 * e], m->tetV[e], p->mu[e], p->lam[e], act_of(p, e));
    }
    for (int t = 0; t < m->nt; ++t) {
        V3<double> xe[3];
        for (int k = 0; k < 3; ++k) xe[k] = load3(&x[3 * m->tri[3 * t + k]]);
        E += tri_energy<double>(xe, &m->triDmInv[4 * t], m->triA[t], p->ktri[t]);
    }
    if (m->ground)
        for (int i = 0; i < m->np; ++i) E += contact_energy(load3(&x[3 * i]), m->plane, p->ke);
    return E;
}

/* One semi-implicit Euler step. */
int oc_step(void* h, const oc_params* p, const double* x, const double* v, double* xo, double* vo) {
    Model* m = static_cast<Model*>(h);
    if (m->status) return m->status;
    std::vector<double> f(3 * (size_t)m->np);
    step(m, p, x, v, xo, vo, f);
    return 0;
}

/* T steps from (x0, v0); xs, vs receive all T+1 states, [(T+1)][np][3]. */
int oc_rollout(void* h, const oc_params* p, const double* x0, const double* v0, int T, double* xs, double* vs) {
    Model* m = static_cast<Model*>(h);
    if (m->status) return m->status;
    size_t n3 = 3 * (size_t)m->np;
    std::vector<double> f(n3);
    std::memcpy(xs, x0, sizeof(double) * n3);
    std::memcpy(vs, v0, sizeof(double) * n3);
    for (int t = 0; t < T; ++t) step(m, p, xs + t * n3, vs + t * n3, xs + (t + 1) * n3, vs + (t + 1) * n3, f);
    return 0;
}

/* T steps keeping only the final state (no trajectory storage). */
int oc_rollout_final(void* h, const oc_params* p, const double* x0, const double* v0, int T, double* xT, double* vT) {
    Model* m = static_cast<Model*>(h);
    if (m->status) return m->status;
    size_t n3 = 3 * (size_t)m->np;
    std::vector<double> f(n3), xa(x0, x0 + n3), va(v0, v0 + n3), xb(n3), vb(n3);
    for (int t = 0; t < T; ++t) {
        step(m, p, xa.data(), va.data(), xb.data(), vb.data(), f);
        xa.swap(xb); va.swap(vb);
    }
    std::memcpy(xT, xa.data(), sizeof(double) * n3);
    std::memcpy(vT, va.data(), sizeof(double) * n3);
    return 0;
}

/* L = (1/np) sum_i |x_i - x*_i|^2; xbar (may be NULL) = dL/dx = 2 (x - x*)/np. */
double oc_loss(void* h, const double* x, const double* target, double* xbar) {
    Model* m = static_cast<Model*>(h);
    double L = 0.0;
    for (int i = 0; i < m->np; ++i)
        for (int c = 0; c < 3; ++c) {
            double d = x[3 * i + c] - target[3 * i + c];
            L += d * d;
            if (xbar) xbar[3 * i + c] = 2.0 * d / m->np;
        }
    return L / m->np;
}

/* (df/dx)^T fbar and (df/dv)^T fbar (written to xbar, vbar), parameter
 * adjoints accumulated into g (may be NULL). */
int oc_force_vjp(void* h, const oc_params* p, const double* x, const double* v, const double* fbar, double* xbar,
                 double* vbar, oc_grads* g) {
    Model* m = static_cast<Model*>(h);
    if (m->status) return m->status;
    std::memset(xbar, 0, sizeof(double) * 3 * m->np);
    std::memset(vbar, 0, sizeof(double) * 3 * m->np);
    force_vjp(m, p, x, v, fbar, xbar, vbar, g);
    return 0;
}

/* Directional derivative of the total force: df = (df/dx) dx + (df/dv) dv
 * + (df/dtheta) dtheta, by a single forward-mode dual pass (tangent slot 0).
 * dp holds the parameter tangents (any pointer may be NULL = zero). */
int oc_force_jvp(void* h, const oc_params* p, const oc_params* dp, const double* x, const double* v,
                 const double* dx, const double* dv, double* df) {
    Model* m = static_cast<Model*>(h);
    if (m->status) return m->status;
    std::vector<V3<Dual> > fd(m->np, zero3<Dual>());
    auto tang = [](double value, double t) { Dual r(value); r.d[0] = t; return r; };
    auto xp = [&](int i) { return mk<Dual>(tang(x[3 * i], dx[3 * i]), tang(x[3 * i + 1], dx[3 * i + 1]), tang(x[3 * i + 2], dx[3 * i + 2])); };
    auto vp = [&](int i) { return mk<Dual>(tang(v[3 * i], dv[3 * i]), tang(v[3 * i + 1], dv[3 * i + 1]), tang(v[3 * i + 2], dv[3 * i + 2])); };
    auto opt = [](const double* a, int i) { return a ? a[i] : 0.0; };
    for (int e = 0; e < m->ne; ++e) {
        const int* id = &m->tet[4 * e];
        V3<Dual> xe[4], fe[4];
        for (int k = 0; k < 4; ++k) xe[k] = xp(id[k]);
        tet_force<Dual>(xe, &m->tetDmInv[9 * e], m->tetV[e], tang(p->mu[e], opt(dp->mu, e)),
                        tang(p->lam[e], opt(dp->lam, e)), tang(act_of(p, e), opt(dp->act, e)), fe);
        for (int k = 0; k < 4; ++k) fd[id[k]] = fd[id[k]] + fe[k];
    }
    for (int t = 0; t < m->nt; ++t) {
        const int* id = &m->tri[3 * t];
        V3<Dual> xe[3], fe[3];
        for (int k = 0; k < 3; ++k) xe[k] = xp(id[k]);
        tri_force<Dual>(xe, &m->triDmInv[4 * t], m->triA[t], tang(p->ktri[t], opt(dp->ktri, t)), fe);
        for (int k = 0; k < 3; ++k) fd[id[k]] = fd[id[k]] + fe[k];
        if (m->air) {
            V3<Dual> ve[3];
            for (int k = 0; k < 3; ++k) ve[k] = vp(id[k]);
            air_force<Dual>(xe, ve, tang(p->kdrag, dp->kdrag), tang(p->klift, dp->klift), fe);
            for (int k = 0; k < 3; ++k) fd[id[k]] = fd[id[k]] + fe[k];
        }
    }
    for (int q = 0; q < m->nh; ++q) {
        const int* id = &m->hinge[4 * q];
        V3<Dual> xe[4], fe[4];
        for (int k = 0; k < 4; ++k) xe[k] = xp(id[k]);
        hinge_force<Dual>(xe, m->phi0[q], tang(p->kb, dp->kb), tang(hact_of(p, q), opt(dp->hact, q)), fe);
        for (int k = 0; k < 4; ++k) fd[id[k]] = fd[id[k]] + fe[k];
    }
    if (m->ground)
        for (int i = 0; i < m->np; ++i)
            fd[i] = fd[i] + contact_force<Dual>(xp(i), vp(i), m->plane, tang(p->ke, dp->ke), tang(p->kd, dp->kd),
                                                tang(p->kf, dp->kf), tang(p->muf, dp->muf));
    for (int i = 0; i < m->np; ++i) {
        df[3 * i] = fd[i].x.d[0];
        df[3 * i + 1] = fd[i].y.d[0];
        df[3 * i + 2] = fd[i].z.d[0];
    }
    return 0;
}

/* One reverse step at state (x, v): (xbp, vbp) = adjoint of the step output,
 * (xbm, vbm) = adjoint of the step input; parameter grads accumulate. */
int oc_step_vjp(void* h, const oc_params* p, const double* x, const double* v, const double* xbp, const double* vbp,
                double* xbm, double* vbm, oc_grads* g) {
    Model* m = static_cast<Model*>(h);
    if (m->status) return m->status;
    std::vector<double> f(3 * (size_t)m->np), fbar(3 * (size_t)m->np);
    step_vjp(m, p, x, v, xbp, vbp, xbm, vbm, g, f, fbar);
    return 0;
}

/* Reverse pass over a stored trajectory (xs, vs of T+1 states), starting from
 * the adjoint of the final state (xbT, vbT).  Writes the adjoint of the
 * initial state into (xb0, vb0) and accumulates parameter grads into g
 * (App. A: the adjoint is carried back one step at a time). */
int oc_backward(void* h, const oc_params* p, const double* xs, const double* vs, int T, const double* xbT,
                const double* vbT, double* xb0, double* vb0, oc_grads* g) {
    Model* m = static_cast<Model*>(h);
    if (m->status) return m->status;
    size_t n3 = 3 * (size_t)m->np;
    std::vector<double> f(n3), fbar(n3), xa(xbT, xbT + n3), va(vbT, vbT + n3), xb(n3), vb(n3);
    for (int t = T - 1; t >= 0; --t) {
        step_vjp(m, p, xs + t * n3, vs + t * n3, xa.data(), va.data(), xb.data(), vb.data(), g, f, fbar);
        xa.swap(xb); va.swap(vb);
    }
    std::memcpy(xb0, xa.data(), sizeof(double) * n3);
    std::memcpy(vb0, va.data(), sizeof(double) * n3);
    return 0;
}

/* ---- single-element entry points (for element-level pins) ---- */

static void unpack(const double* a, int n, V3<double>* x) { for (int k = 0; k < n; ++k) x[k] = load3(&a[3 * k]); }
static void pack(double* a, int n, const V3<double>* x) { for (int k = 0; k < n; ++k) store3(&a[3 * k], x[k]); }

/* Tet: x, X are [4][3]. Returns V (rest volume). */
double oc_tet_force1(const double* x, const double* X, double mu, double lam, double act, double* f) {
    V3<double> xe[4], Xe[4], fe[4];
    double DmInv[9];
    unpack(x, 4, xe); unpack(X, 4, Xe);
    double V = tet_rest(Xe, DmInv) / 6.0;
    tet_force<double>(xe, DmInv, V, mu, lam, act, fe);
    pack(f, 4, fe);
    return V;
}
double oc_tet_energy1(const double* x, const double* X, double mu, double lam, double act) {
    V3<double> xe[4], Xe[4];
    double DmInv[9];
    unpack(x, 4, xe); unpack(X, 4, Xe);
    double V = tet_rest(Xe, DmInv) / 6.0;
    return tet_energy<double>(xe, DmInv, V, mu, lam, act);
}
double oc_tri_force1(const double* x, const double* X, double k, double* f) {
    V3<double> xe[3], Xe[3], fe[3];
    double DmInv[4];
    unpack(x, 3, xe); unpack(X, 3, Xe);
    double A = tri_rest(Xe, DmInv);
    tri_force<double>(xe, DmInv, A, k, fe);
    pack(f, 3, fe);
    return A;
}
double oc_tri_energy1(const double* x, const double* X, double k) {
    V3<double> xe[3], Xe[3];
    double DmInv[4];
    unpack(x, 3, xe); unpack(X, 3, Xe);
    double A = tri_rest(Xe, DmInv);
    return tri_energy<double>(xe, DmInv, A, k);
}
double oc_hinge_angle1(const double* x) {
    V3<double> xe[4];
    unpack(x, 4, xe);
    return hinge_angle<double>(xe);
}
void oc_air_force1(const double* x, const double* v, double kd, double kl, double* f) {
    V3<double> xe[3], ve[3], fe[3];
    for (int k = 0; k < 3; ++k) {
        xe[k] = load3(&x[3 * k]);
        ve[k] = load3(&v[3 * k]);
    }
    air_force<double>(xe, ve, kd, kl, fe);
    for (int k = 0; k < 3; ++k) {
        f[3 * k] = fe[k].x;
        f[3 * k + 1] = fe[k].y;
        f[3 * k + 2] = fe[k].z;
    }
}

void oc_hinge_force1(const double* x, double phi0, double kb, double act, double* f) {
    V3<double> xe[4], fe[4];
    unpack(x, 4, xe);
    hinge_force<double>(xe, phi0, kb, act, fe);
    pack(f, 4, fe);
}
void oc_contact_force1(const double* x, const double* v, const double* plane, double ke, double kd, double kf,
                       double muf, double* f) {
    V3<double> fc = contact_force<double>(load3(x), load3(v), plane, ke, kd, kf, muf);
    store3(f, fc);
}

}  // extern "C"

/* ====================================================================== */
/* Rigid bodies (App. A.1 "Rigid bodies" and "Contact")                    */
/* ====================================================================== */
/* State s = [x (3), r (4) = (w, i, j, k), v (3), omega (3)]: centre-of-mass
 * position, orientation quaternion (body to world), linear and angular velocity
 * (world frame).  Parameters: mass m, body-frame inertia about the centre of mass
 * I = [Ixx, Iyy, Izz, Ixy, Ixz, Iyz], contact [ke, kd, kf, muf].  Vertices p_k are
 * body-frame positions relative to the centre of mass; each is tested against
 * the ground plane with the particle contact model. */
namespace {

/* Rotation matrix (row-major) of a unit quaternion. */
template <class S> void quat_rot(const S q[4], S R[9]) {
    const S w = q[0], a = q[1], b = q[2], c = q[3];
    R[0] = 1.0 - 2.0 * (b * b + c * c); R[1] = 2.0 * (a * b - w * c);       R[2] = 2.0 * (a * c + w * b);
    R[3] = 2.0 * (a * b + w * c);       R[4] = 1.0 - 2.0 * (a * a + c * c); R[5] = 2.0 * (b * c - w * a);
    R[6] = 2.0 * (a * c - w * b);       R[7] = 2.0 * (b * c + w * a);       R[8] = 1.0 - 2.0 * (a * a + b * b);
}

template <class S> V3<S> mat_vec(const S M[9], const V3<S>& v) {
    return mk<S>(M[0] * v.x + M[1] * v.y + M[2] * v.z, M[3] * v.x + M[4] * v.y + M[5] * v.z,
                 M[6] * v.x + M[7] * v.y + M[8] * v.z);
}

/* One semi-implicit Euler step of one rigid body (App. A.2 applied to the
 * Newton-Euler equations): forces and torques at the step's start state,
 *   v+ = v + dt (F / m + g)
 *   omega+ = omega + dt Iw^-1 (tau - omega x (Iw omega)),  Iw = R I R^T
 *   x+ = x + dt v+,   r+ = normalise(r + dt/2 [0, omega+] (x) r). */
template <class S>
void rigid_step(const S s[13], S m, const S I[6], const S c[4], const double* p, int nv, const double g[3],
                const double plane[4], int ground, double dt, S out[13]) {
    const V3<S> x = mk<S>(s[0], s[1], s[2]);
    const S* r = &s[3];
    const V3<S> v = mk<S>(s[7], s[8], s[9]);
    const V3<S> w = mk<S>(s[10], s[11], s[12]);
    S R[9];
    quat_rot<S>(r, R);
    V3<S> F = zero3<S>(), tau = zero3<S>();
    if (ground)
        for (int k = 0; k < nv; ++k) {
            const V3<S> pk = mk<S>(S(p[3 * k]), S(p[3 * k + 1]), S(p[3 * k + 2]));
            const V3<S> a = mat_vec<S>(R, pk);
            const V3<S> f = contact_force<S>(x + a, v + cross(w, a), plane, c[0], c[1], c[2], c[3]);
            F = F + f;
            tau = tau + cross(a, f);
        }
    /* Iw = R Ib R^T */
    const S Ib[9] = {I[0], I[3], I[4], I[3], I[1], I[5], I[4], I[5], I[2]};
    S T1[9], Iw[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            S acc = S(0.0);
            for (int k = 0; k < 3; ++k) acc = acc + R[3 * i + k] * Ib[3 * k + j];
            T1[3 * i + j] = acc;
        }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            S acc = S(0.0);
            for (int k = 0; k < 3; ++k) acc = acc + T1[3 * i + k] * R[3 * j + k];
            Iw[3 * i + j] = acc;
        }
    const V3<S> L = mat_vec<S>(Iw, w);
    const V3<S> h = tau - cross(w, L);
    /* alpha = Iw^-1 h by the adjugate */
    const S det = Iw[0] * (Iw[4] * Iw[8] - Iw[5] * Iw[7]) - Iw[1] * (Iw[3] * Iw[8] - Iw[5] * Iw[6]) +
                  Iw[2] * (Iw[3] * Iw[7] - Iw[4] * Iw[6]);
    S inv[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const int r1 = (j + 1) % 3, r2 = (j + 2) % 3, c1 = (i + 1) % 3, c2 = (i + 2) % 3;
            inv[3 * i + j] = (Iw[3 * r1 + c1] * Iw[3 * r2 + c2] - Iw[3 * r1 + c2] * Iw[3 * r2 + c1]) / det;
        }
    const V3<S> alpha = mat_vec<S>(inv, h);
    const V3<S> vn = v + (F * (S(1.0) / m) + mk<S>(S(g[0]), S(g[1]), S(g[2]))) * dt;
    const V3<S> wn = w + alpha * dt;
    const V3<S> xn = x + vn * dt;
    /* [0, wn] (x) r = [-wn . u, r0 wn + wn x u], u = (r1, r2, r3) */
    const V3<S> u = mk<S>(r[1], r[2], r[3]);
    const S q0 = r[0] - 0.5 * dt * dot(wn, u);
    const V3<S> qv = u + (wn * r[0] + cross(wn, u)) * (0.5 * dt);
    const S qn = sqrt(q0 * q0 + dot(qv, qv));
    out[0] = xn.x; out[1] = xn.y; out[2] = xn.z;
    out[3] = q0 / qn; out[4] = qv.x / qn; out[5] = qv.y / qn; out[6] = qv.z / qn;
    out[7] = vn.x; out[8] = vn.y; out[9] = vn.z;
    out[10] = wn.x; out[11] = wn.y; out[12] = wn.z;
}

/* Mean squared distance of the body's world vertices to target points. */
template <class S> S rigid_loss(const S s[13], const double* p, int nv, const double* target) {
    S R[9];
    quat_rot<S>(&s[3], R);
    S L = S(0.0);
    for (int k = 0; k < nv; ++k) {
        const V3<S> a = mat_vec<S>(R, mk<S>(S(p[3 * k]), S(p[3 * k + 1]), S(p[3 * k + 2])));
        const V3<S> d = mk<S>(s[0] + a.x - target[3 * k], s[1] + a.y - target[3 * k + 1], s[2] + a.z - target[3 * k + 2]);
        L = L + dot(d, d);
    }
    return L / double(nv);
}

}  // namespace

extern "C" {

/* One rigid step; s, out [13]; I [6]; c [4]; p [nv][3]; g [3]; plane [4]. */
void oc_rigid_step(int nv, const double* p, const double* s, double m, const double* I, const double* c,
                   const double* g, const double* plane, int ground, double dt, double* out) {
    rigid_step<double>(s, m, I, c, p, nv, g, plane, ground, dt, out);
}

/* Reverse mode of one rigid step by forward-mode duals: the 24 inputs
 * [s (13), m, I (6), c (4)] are seeded in two passes of up to ND tangents; each
 * input's adjoint is sum_o out_bar[o] d out_o / d input.  Adds into s_bar [13],
 * m_bar [1], I_bar [6], c_bar [4]. */
void oc_rigid_step_vjp(int nv, const double* p, const double* s, double m, const double* I, const double* c,
                       const double* g, const double* plane, int ground, double dt, const double* out_bar,
                       double* s_bar, double* m_bar, double* I_bar, double* c_bar) {
    const int NIN = 24;
    double in[NIN];
    for (int k = 0; k < 13; ++k) in[k] = s[k];
    in[13] = m;
    for (int k = 0; k < 6; ++k) in[14 + k] = I[k];
    for (int k = 0; k < 4; ++k) in[20 + k] = c[k];
    double grad[NIN];
    for (int first = 0; first < NIN; first += ND) {
        Dual z[NIN];
        for (int k = 0; k < NIN; ++k) {
            z[k] = Dual(in[k]);
            if (k >= first && k < first + ND) z[k].d[k - first] = 1.0;
        }
        Dual out[13];
        rigid_step<Dual>(z, z[13], &z[14], &z[20], p, nv, g, plane, ground, dt, out);
        for (int k = first; k < NIN && k < first + ND; ++k) {
            double acc = 0.0;
            for (int o = 0; o < 13; ++o) acc += out_bar[o] * out[o].d[k - first];
            grad[k] = acc;
        }
    }
    for (int k = 0; k < 13; ++k) s_bar[k] += grad[k];
    m_bar[0] += grad[13];
    for (int k = 0; k < 6; ++k) I_bar[k] += grad[14 + k];
    for (int k = 0; k < 4; ++k) c_bar[k] += grad[20 + k];
}

/* Vertex loss of one body and its gradient with respect to the state (s_bar [13],
 * overwritten; only x and r enter). */
double oc_rigid_loss(int nv, const double* p, const double* s, const double* target, double* s_bar) {
    Dual z[13];
    for (int k = 0; k < 13; ++k) {
        z[k] = Dual(s[k]);
        if (k < ND) z[k].d[k] = 1.0;
    }
    Dual L = rigid_loss<Dual>(z, p, nv, target);
    if (s_bar)
        for (int k = 0; k < 13; ++k) s_bar[k] = L.d[k];
    return L.v;
}

}  // extern "C"
