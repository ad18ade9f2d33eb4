/*
 * FP64 CPU oracle for the fast explicit dynamics FEM (FED-FEM) of
 * Zhang & Chauhan, "Fast explicit dynamics finite element algorithm for
 * transient heat transfer" (arXiv 1909.03355).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU library is checked against.  Nothing in the product path links it; it
 * shares no code, header or table with the GPU library.
 *
 * It follows the paper's three stages (Sec. 3.5) literally:
 *   pre-computation  - per element det J and B, G = 8 det(J) B^T (hexahedra,
 *                      one centre Gauss point, Eq. 17, 19) or G = V B^T
 *                      (tetrahedra, Eq. 18, 19); lumped thermal mass (Sec. 3.1)
 *   time stepping    - element loads F_e = G D(T) B T_e (Eq. 20), summed at
 *                      the nodes without a global K (Eq. 10-11), surface loads
 *                      Q (Eqs. 4, 5, 7), explicit update (Eq. 15-16), then the
 *                      essential condition (Eq. 3) for the next step.
 * Readings of the paper used here (where it is garbled or silent):
 *   - F in Eq. 9-16 is read as the conductive heat INTO the nodes, -K T, so
 *     the update is T += dt (Q - K T) / C  (K = sum of B^T D B dV is PSD).
 *   - convection adds -h A (T - Ta) into a node (the physical sign, Eq. 7's).
 *   - surface loads are lumped to the face nodes with area |f| / n_f.
 *   - c(T) is evaluated at the node; the conductivity factor of D(T) is
 *     evaluated at every node of the element and the nodal values averaged
 *     (Sec. 4.2.2), which for a linear k(T) equals its value at the element's
 *     mean temperature.
 *   - the lumped mass uses the exact element volume (2x2x2 Gauss for a
 *     trilinear hexahedron, which is exact), stiffness uses 8 det J(0).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const int HEX_S[8][3] = {
    {-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
    {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};

static double det3(double J[3][3]) {
  return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
         J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
         J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

/* Inverse of a 3x3 matrix by the adjugate. */
static void inv3(double J[3][3], double d, double R[3][3]) {
  R[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / d;
  R[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / d;
  R[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / d;
  R[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / d;
  R[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / d;
  R[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / d;
  R[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / d;
  R[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / d;
  R[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / d;
}

/* Derivatives of the trilinear shape functions N_a = (1+s_a.xi)(1+s_a.eta)(1+s_a.zeta)/8
 * with respect to the natural coordinates, at natural point p. */
static void hex_dN(const double p[3], double dN[8][3]) {
  for (int a = 0; a < 8; a++) {
    double sx = HEX_S[a][0], sy = HEX_S[a][1], sz = HEX_S[a][2];
    dN[a][0] = sx * (1 + sy * p[1]) * (1 + sz * p[2]) / 8.0;
    dN[a][1] = sy * (1 + sx * p[0]) * (1 + sz * p[2]) / 8.0;
    dN[a][2] = sz * (1 + sx * p[0]) * (1 + sy * p[1]) / 8.0;
  }
}

/* J[i][j] = d x_i / d xi_j = sum_a X_a,i dN_a/dxi_j */
static void hex_jac(double X[8][3], double dN[8][3], double J[3][3]) {
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double s = 0;
      for (int a = 0; a < 8; a++) s += X[a][i] * dN[a][j];
      J[i][j] = s;
    }
}

/* Solve A X = I for a 4x4 matrix by Gauss-Jordan elimination with partial
 * pivoting; returns det(A). */
static double inv4(double A[4][4], double X[4][4]) {
  double M[4][8];
  for (int i = 0; i < 4; i++)
    for (int j = 0; j < 4; j++) {
      M[i][j] = A[i][j];
      M[i][4 + j] = (i == j) ? 1.0 : 0.0;
    }
  double det = 1.0;
  for (int c = 0; c < 4; c++) {
    int piv = c;
    for (int r = c + 1; r < 4; r++)
      if (fabs(M[r][c]) > fabs(M[piv][c])) piv = r;
    if (M[piv][c] == 0.0) return 0.0;
    if (piv != c) {
      for (int j = 0; j < 8; j++) {
        double t = M[c][j];
        M[c][j] = M[piv][j];
        M[piv][j] = t;
      }
      det = -det;
    }
    double p = M[c][c];
    det *= p;
    for (int j = 0; j < 8; j++) M[c][j] /= p;
    for (int r = 0; r < 4; r++) {
      if (r == c) continue;
      double f = M[r][c];
      for (int j = 0; j < 8; j++) M[r][j] -= f * M[c][j];
    }
  }
  for (int i = 0; i < 4; i++)
    for (int j = 0; j < 4; j++) X[i][j] = M[i][4 + j];
  return det;
}

/*
 * Pre-computation (Sec. 3.5 (i).2): per element B (3 x ne, row-major at
 * B[(e*3+i)*ne + a]), the stiffness weight W (8 det J(0) for hexahedra, V
 * for tetrahedra), the exact volume V and the orientation determinant.
 * Returns the number of inverted or degenerate elements.
 */
int64_t orc_geometry(int ne, int64_t E, const double *x, const double *y,
                     const double *z, const int32_t *conn, double *B, double *W,
                     double *V, double *detJ0) {
  int64_t bad = 0;
  for (int64_t e = 0; e < E; e++) {
    if (ne == 8) {
      double X[8][3], dN[8][3], J[3][3], Ji[3][3];
      for (int a = 0; a < 8; a++) {
        int32_t k = conn[(int64_t)a * E + e];
        X[a][0] = x[k];
        X[a][1] = y[k];
        X[a][2] = z[k];
      }
      const double zero[3] = {0, 0, 0};
      hex_dN(zero, dN);
      hex_jac(X, dN, J);
      double d = det3(J);
      detJ0[e] = d;
      if (!(d > 0)) {
        bad++;
        d = (d == 0) ? 1.0 : d;
      }
      inv3(J, d, Ji);
      /* B = J^{-T} dN^T:  B[i][a] = sum_j Ji[j][i] dN[a][j] */
      for (int i = 0; i < 3; i++)
        for (int a = 0; a < 8; a++) {
          double s = 0;
          for (int j = 0; j < 3; j++) s += Ji[j][i] * dN[a][j];
          B[(e * 3 + i) * 8 + a] = s;
        }
      W[e] = 8.0 * detJ0[e];
      /* exact volume of the trilinear map: 2x2x2 Gauss, unit weights */
      double vol = 0;
      const double g = 1.0 / sqrt(3.0);
      for (int q = 0; q < 8; q++) {
        double p[3] = {HEX_S[q][0] * g, HEX_S[q][1] * g, HEX_S[q][2] * g};
        double dNq[8][3], Jq[3][3];
        hex_dN(p, dNq);
        hex_jac(X, dNq, Jq);
        vol += det3(Jq);
      }
      V[e] = vol;
    } else {
      /* linear tetrahedron: N_a(x) = C[0][a] + C[1][a] x + C[2][a] y + C[3][a] z
       * with C = P^{-1}, P rows [1 x_a y_a z_a]; B[i][a] = C[1+i][a]. */
      double P[4][4], C[4][4];
      for (int a = 0; a < 4; a++) {
        int32_t k = conn[(int64_t)a * E + e];
        P[a][0] = 1.0;
        P[a][1] = x[k];
        P[a][2] = y[k];
        P[a][3] = z[k];
      }
      double d = inv4(P, C);
      detJ0[e] = d;
      if (d == 0.0) bad++;
      for (int i = 0; i < 3; i++)
        for (int a = 0; a < 4; a++) B[(e * 3 + i) * 4 + a] = C[1 + i][a];
      V[e] = fabs(d) / 6.0;
      W[e] = V[e];
    }
  }
  return bad;
}

/*
 * Uniform-gradient (mean) hexahedron, an alternative to the centre point of
 * Eq. 17 for distorted hexahedra: B_e is the gradient operator averaged over
 * the element, Bbar = (1/V) integral of B dV, and W = V, so K_e = V Bbar^T D
 * Bbar.  B det J is a polynomial of degree <= 3 in each natural coordinate
 * (cofactors of J times the shape-function derivatives), so the 2x2x2 Gauss
 * rule integrates it exactly.  By the divergence theorem Bbar reproduces any
 * linear field exactly on every hexahedron.  Same outputs and return value as
 * orc_geometry (hexahedra only).
 */
int64_t orc_geometry_mean(int64_t E, const double *x, const double *y, const double *z,
                          const int32_t *conn, double *B, double *W, double *V, double *detJ0) {
  int64_t bad = 0;
  const double g = 1.0 / sqrt(3.0);
  for (int64_t e = 0; e < E; e++) {
    double X[8][3];
    for (int a = 0; a < 8; a++) {
      int32_t k = conn[(int64_t)a * E + e];
      X[a][0] = x[k];
      X[a][1] = y[k];
      X[a][2] = z[k];
    }
    double dN0[8][3], J0[3][3];
    const double zero[3] = {0, 0, 0};
    hex_dN(zero, dN0);
    hex_jac(X, dN0, J0);
    detJ0[e] = det3(J0);
    if (!(detJ0[e] > 0)) bad++;
    double S[3][8] = {{0}}, vol = 0;
    for (int q = 0; q < 8; q++) {
      double p[3] = {HEX_S[q][0] * g, HEX_S[q][1] * g, HEX_S[q][2] * g};
      double dN[8][3], J[3][3], Ji[3][3];
      hex_dN(p, dN);
      hex_jac(X, dN, J);
      double d = det3(J);
      if (!(d > 0)) bad++;
      vol += d;
      inv3(J, d == 0 ? 1.0 : d, Ji);
      /* B det J at the point: B[i][a] = sum_j Ji[j][i] dN[a][j] */
      for (int i = 0; i < 3; i++)
        for (int a = 0; a < 8; a++) {
          double t = 0;
          for (int j = 0; j < 3; j++) t += Ji[j][i] * dN[a][j];
          S[i][a] += t * d;
        }
    }
    V[e] = vol;
    W[e] = vol;
    for (int i = 0; i < 3; i++)
      for (int a = 0; a < 8; a++) B[(e * 3 + i) * 8 + a] = S[i][a] / (vol == 0 ? 1.0 : vol);
  }
  return bad;
}

/* Area of every boundary face: planar triangles by the cross product,
 * bilinear quadrilaterals by 2x2 Gauss quadrature of |x_u x x_v|. */
void orc_face_areas(int nfn, int64_t nf, const double *x, const double *y,
                    const double *z, const int32_t *faces, double *area) {
  for (int64_t f = 0; f < nf; f++) {
    double X[4][3];
    for (int b = 0; b < nfn; b++) {
      int32_t k = faces[f * nfn + b];
      X[b][0] = x[k];
      X[b][1] = y[k];
      X[b][2] = z[k];
    }
    if (nfn == 3) {
      double u[3], v[3];
      for (int i = 0; i < 3; i++) {
        u[i] = X[1][i] - X[0][i];
        v[i] = X[2][i] - X[0][i];
      }
      double c0 = u[1] * v[2] - u[2] * v[1];
      double c1 = u[2] * v[0] - u[0] * v[2];
      double c2 = u[0] * v[1] - u[1] * v[0];
      area[f] = 0.5 * sqrt(c0 * c0 + c1 * c1 + c2 * c2);
    } else {
      static const double su[4] = {-1, 1, 1, -1}, sv[4] = {-1, -1, 1, 1};
      const double g = 1.0 / sqrt(3.0);
      double A = 0;
      for (int q = 0; q < 4; q++) {
        double pu = su[q] * g, pv = sv[q] * g;
        double xu[3] = {0, 0, 0}, xv[3] = {0, 0, 0};
        for (int b = 0; b < 4; b++) {
          double dnu = su[b] * (1 + sv[b] * pv) / 4.0;
          double dnv = sv[b] * (1 + su[b] * pu) / 4.0;
          for (int i = 0; i < 3; i++) {
            xu[i] += X[b][i] * dnu;
            xv[i] += X[b][i] * dnv;
          }
        }
        double c0 = xu[1] * xv[2] - xu[2] * xv[1];
        double c1 = xu[2] * xv[0] - xu[0] * xv[2];
        double c2 = xu[0] * xv[1] - xu[1] * xv[0];
        A += sqrt(c0 * c0 + c1 * c1 + c2 * c2);
      }
      area[f] = A;
    }
  }
}

/* Everything one explicit run needs; arrays are per element (E), per node
 * (N), per face (nf) as named.  Dk is the element conductivity tensor, 6 rows
 * (xx, yy, zz, xy, yz, xz) of length E, with any per-element factor folded in;
 * D_e(T) = Dk * s_e with s_e the mean over the element's nodes of s0 + s1 T_a.
 * c(T) = c0 + c1 * T. */
typedef struct {
  int32_t ne, nfn;
  int64_t N, E, nf, npt, ndir;
  const int32_t *conn;
  const double *B, *W, *V;
  const double *rho, *c0, *c1, *s0, *s1, *Dk;
  const int32_t *faces;
  const double *farea, *fh, *fTa, *feps, *fq;
  const int32_t *pt_nodes;
  const double *pt_W;
  const int32_t *dir_nodes;
  const double *dir_T;
  const double *dt; /* per node */
  double Tz, sigma;
  /* optional piecewise-linear multiplier tables (n points, T increasing):
   * with nkt > 0, the nodal values fk(T_a) replace s0 + s1 T_a; with nct > 0,
   * c_e(T) = c0_e * fc(T) replaces c0 + c1 T */
  int32_t nkt, nct;
  const double *kt_T, *kt_f, *ct_T, *ct_f;
  /* optional hourglass control of the uniform-gradient hexahedron: per element
   * the four vectors gamma (4 x 8) and kappa (see orc_hourglass); NULL = off */
  const double *hg_G, *hg_k;
} orc_problem;

/* Piecewise-linear interpolation in a table, constant beyond its ends;
 * *slope receives the derivative (0 beyond the ends; the left segment's at a
 * breakpoint). */
static double table_eval(int32_t n, const double *Tt, const double *f, double T, double *slope) {
  if (T <= Tt[0]) {
    *slope = 0.0;
    return f[0];
  }
  if (T >= Tt[n - 1]) {
    *slope = 0.0;
    return f[n - 1];
  }
  int i = 1;
  while (T > Tt[i]) i++;
  const double h = Tt[i] - Tt[i - 1];
  *slope = (f[i] - f[i - 1]) / h;
  return f[i - 1] + (T - Tt[i - 1]) / h * (f[i] - f[i - 1]);
}

/* conductivity factor of element e's material at one node temperature T
 * (s0 + s1 T, or the k table) and its derivative */
static double kfac_node(const orc_problem *P, int64_t e, double T, double *ds) {
  if (P->nkt > 0) return table_eval(P->nkt, P->kt_T, P->kt_f, T, ds);
  *ds = P->s1[e];
  return P->s0[e] + P->s1[e] * T;
}

/* Element conductivity factor (Sec. 4.2.2): the property is evaluated at each
 * node of the element from that node's temperature, and the nodal values are
 * averaged for the element-level calculation.  ds[a] receives
 * d s_e / d T_a = (d s / d T)(T_a) / n_e. */
static double kfac(const orc_problem *P, int64_t e, const double *Te, double *ds) {
  double s = 0;
  for (int a = 0; a < P->ne; a++) {
    double d;
    s += kfac_node(P, e, Te[a], &d);
    ds[a] = d / P->ne;
  }
  return s / P->ne;
}

/* specific heat c_e(T) and its derivative */
static double cfun(const orc_problem *P, int64_t e, double T, double *dc) {
  if (P->nct > 0) {
    double sl;
    const double v = table_eval(P->nct, P->ct_T, P->ct_f, T, &sl);
    *dc = P->c0[e] * sl;
    return P->c0[e] * v;
  }
  *dc = P->c1[e];
  return P->c0[e] + P->c1[e] * T;
}

/* Element load F_e = G D_e B T_e with G = W B^T (Eq. 19-20) and D_e from the
 * nodal average of the conductivity factor (kfac). */
static void element_load(const orc_problem *P, int64_t e, const double *T, double *Fe) {
  int ne = P->ne;
  int64_t E = P->E;
  double Te[8], ds[8];
  for (int a = 0; a < ne; a++) Te[a] = T[P->conn[(int64_t)a * E + e]];
  const double s = kfac(P, e, Te, ds);
  const double *Dk = P->Dk;
  double D[3][3];
  D[0][0] = Dk[0 * E + e] * s;
  D[1][1] = Dk[1 * E + e] * s;
  D[2][2] = Dk[2 * E + e] * s;
  D[0][1] = D[1][0] = Dk[3 * E + e] * s;
  D[1][2] = D[2][1] = Dk[4 * E + e] * s;
  D[0][2] = D[2][0] = Dk[5 * E + e] * s;
  const double *Be = P->B + e * 3 * ne;
  double g[3], q[3];
  for (int i = 0; i < 3; i++) {
    g[i] = 0;
    for (int a = 0; a < ne; a++) g[i] += Be[i * ne + a] * Te[a];
  }
  for (int i = 0; i < 3; i++) q[i] = D[i][0] * g[0] + D[i][1] * g[1] + D[i][2] * g[2];
  for (int a = 0; a < ne; a++) {
    double s2 = 0;
    for (int i = 0; i < 3; i++) s2 += P->W[e] * Be[i * ne + a] * q[i];
    Fe[a] = s2;
  }
  if (P->hg_k) {
    /* s kappa sum_alpha (gamma_alpha . T_e) gamma_alpha */
    const double *G = P->hg_G + e * 32;
    for (int al = 0; al < 4; al++) {
      double c = 0;
      for (int a = 0; a < 8; a++) c += G[al * 8 + a] * Te[a];
      for (int a = 0; a < 8; a++) Fe[a] += s * P->hg_k[e] * c * G[al * 8 + a];
    }
  }
}

/* Hourglass control of the uniform-gradient hexahedron (not in the paper: the
 * scalar-field form of Flanagan and Belytschko's orthogonal hourglass control,
 * 1981).  With the hourglass patterns h_1 = eta zeta, h_2 = zeta xi,
 * h_3 = xi eta, h_4 = xi eta zeta of the nodes' natural signs, b_i the rows of
 * the mean gradient operator (B, 3 x 8) and x_i the nodal coordinates,
 *   gamma_alpha = (h_alpha - sum_i (h_alpha . x_i) b_i) / 8
 * vanishes on every linear field (b reproduces its gradient), and the element
 * adds K_hg = kappa sum_alpha gamma_alpha gamma_alpha^T to its conductance,
 *   kappa = eps (tr Dk / 3) V sum_a |b_a|^2,
 * scaled by the conductivity factor s_e like the rest of the element.  On
 * a cube of side h, gamma_alpha = h_alpha / 8 and kappa = 1.5 eps k h.
 * G receives gamma (E x 4 x 8), kap kappa (E). */
void orc_hourglass(int64_t E, const double *x, const double *y, const double *z,
                   const int32_t *conn, const double *B, const double *V, const double *Dk,
                   double eps, double *G, double *kap) {
  for (int64_t e = 0; e < E; e++) {
    double X[8][3];
    for (int a = 0; a < 8; a++) {
      const int32_t k = conn[(int64_t)a * E + e];
      X[a][0] = x[k];
      X[a][1] = y[k];
      X[a][2] = z[k];
    }
    const double *Be = B + e * 24;
    double bb = 0;
    for (int i = 0; i < 24; i++) bb += Be[i] * Be[i];
    kap[e] = eps * (Dk[0 * E + e] + Dk[1 * E + e] + Dk[2 * E + e]) / 3.0 * V[e] * bb;
    for (int al = 0; al < 4; al++) {
      double h[8], hx[3] = {0, 0, 0};
      for (int a = 0; a < 8; a++) {
        const double sx = HEX_S[a][0], sy = HEX_S[a][1], sz = HEX_S[a][2];
        h[a] = al == 0 ? sy * sz : al == 1 ? sz * sx : al == 2 ? sx * sy : sx * sy * sz;
        for (int i = 0; i < 3; i++) hx[i] += h[a] * X[a][i];
      }
      for (int a = 0; a < 8; a++)
        G[e * 32 + al * 8 + a] =
            (h[a] - (hx[0] * Be[0 * 8 + a] + hx[1] * Be[1 * 8 + a] + hx[2] * Be[2 * 8 + a])) / 8.0;
    }
  }
}

/* Threads of the element loop (OpenMP): the count in use, and a new count
 * (n >= 1) for the timed single-thread baseline. */
int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* Net nodal conductive load F = sum_e F_e (summed in element order) and the
 * lumped heat capacity C_k = sum_{e owns k} rho_e V_e / n_e * c_e(T_k). */
void orc_loads(const orc_problem *P, const double *T, double *Fe, double *F, double *C) {
  int ne = P->ne;
  int64_t E = P->E;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < E; e++) element_load(P, e, T, Fe + e * ne);
  memset(F, 0, sizeof(double) * P->N);
  memset(C, 0, sizeof(double) * P->N);
  for (int64_t e = 0; e < E; e++)
    for (int a = 0; a < ne; a++) {
      int32_t k = P->conn[(int64_t)a * E + e];
      F[k] += Fe[e * ne + a];
      double dc;
      C[k] += P->rho[e] * P->V[e] / ne * cfun(P, e, T[k], &dc);
    }
}

/* Net nodal surface heat input Q (Eqs. 4, 5, 7 with the readings above), plus
 * concentrated nodal loads. */
void orc_surface(const orc_problem *P, const double *T, double *Q) {
  memset(Q, 0, sizeof(double) * P->N);
  for (int64_t i = 0; i < P->npt; i++) Q[P->pt_nodes[i]] += P->pt_W[i];
  for (int64_t f = 0; f < P->nf; f++) {
    double share = P->farea[f] / P->nfn;
    for (int b = 0; b < P->nfn; b++) {
      int32_t k = P->faces[f * P->nfn + b];
      double conv = -P->fh[f] * (T[k] - P->fTa[f]);
      double rad = -P->sigma * P->feps[f] *
                   (pow(T[k] - P->Tz, 4) - pow(P->fTa[f] - P->Tz, 4));
      Q[k] += share * (conv + rad + P->fq[f]);
    }
  }
}

/* nsteps explicit steps in place on T (Eq. 16, then Eq. 3).  Work arrays:
 * Fe[E*ne], F, C, Q, Tn [N].  If hist is non-null, hist[(n)*N + k] receives
 * T after n steps for n = 0..nsteps. */
void orc_run(const orc_problem *P, double *T, int64_t nsteps, double *Fe, double *F,
             double *C, double *Q, double *Tn, double *hist) {
  int64_t N = P->N;
  if (hist) memcpy(hist, T, sizeof(double) * N);
  for (int64_t n = 0; n < nsteps; n++) {
    orc_loads(P, T, Fe, F, C);
    orc_surface(P, T, Q);
    for (int64_t k = 0; k < N; k++) Tn[k] = T[k] + P->dt[k] * (Q[k] - F[k]) / C[k];
    for (int64_t i = 0; i < P->ndir; i++) Tn[P->dir_nodes[i]] = P->dir_T[i];
    memcpy(T, Tn, sizeof(double) * N);
    if (hist) memcpy(hist + (n + 1) * N, T, sizeof(double) * N);
  }
}

/* orc_run with concentrated loads that change from step to step (a moving or
 * time-varying source; the explicit scheme of Sec. 3.1 evaluates the loads at
 * the start of each step): step n, counted from step0, takes its loads from row
 * (step0 + n) mod nrows of Wrows (nrows x npt, row-major) instead of pt_W. */
void orc_run_sched(const orc_problem *P, double *T, int64_t nsteps, int64_t step0, int64_t nrows,
                   const double *Wrows, double *Fe, double *F, double *C, double *Q, double *Tn,
                   double *hist) {
  orc_problem Pn = *P;
  if (hist) memcpy(hist, T, sizeof(double) * P->N);
  for (int64_t n = 0; n < nsteps; n++) {
    Pn.pt_W = Wrows + ((step0 + n) % nrows) * P->npt;
    orc_run(&Pn, T, 1, Fe, F, C, Q, Tn, NULL);
    if (hist) memcpy(hist + (n + 1) * P->N, T, sizeof(double) * P->N);
  }
}

/* s K0_e v_e = W B^T (s Dk) B v_e: the element operator at a given factor s
 * applied to the nodal values v (the adjoint needs it with s taken from T^n
 * while v is the adjoint field). */
static void element_apply(const orc_problem *P, int64_t e, const double *v, double s,
                          double *out) {
  int ne = P->ne;
  int64_t E = P->E;
  double ve[8];
  for (int a = 0; a < ne; a++) ve[a] = v[P->conn[(int64_t)a * E + e]];
  const double *Dk = P->Dk;
  double D[3][3];
  D[0][0] = Dk[0 * E + e] * s;
  D[1][1] = Dk[1 * E + e] * s;
  D[2][2] = Dk[2 * E + e] * s;
  D[0][1] = D[1][0] = Dk[3 * E + e] * s;
  D[1][2] = D[2][1] = Dk[4 * E + e] * s;
  D[0][2] = D[2][0] = Dk[5 * E + e] * s;
  const double *Be = P->B + e * 3 * ne;
  double g[3], q[3];
  for (int i = 0; i < 3; i++) {
    g[i] = 0;
    for (int a = 0; a < ne; a++) g[i] += Be[i * ne + a] * ve[a];
  }
  for (int i = 0; i < 3; i++) q[i] = D[i][0] * g[0] + D[i][1] * g[1] + D[i][2] * g[2];
  for (int a = 0; a < ne; a++) {
    double s2 = 0;
    for (int i = 0; i < 3; i++) s2 += P->W[e] * Be[i * ne + a] * q[i];
    out[a] = s2;
  }
  if (P->hg_k) {
    const double *G = P->hg_G + e * 32;
    for (int al = 0; al < 4; al++) {
      double c = 0;
      for (int a = 0; a < 8; a++) c += G[al * 8 + a] * ve[a];
      for (int a = 0; a < 8; a++) out[a] += s * P->hg_k[e] * c * G[al * 8 + a];
    }
  }
}

/*
 * Discrete adjoint of orc_run (not in the paper: the exact transpose of its
 * explicit recursion).  One step, for a node k that is not Dirichlet, is
 *   T'_k = T_k + dt_k r_k(T) / C_k(T_k),   r = Q(T) - F(T),
 * with F_e = s_e K0_e T_e (s_e = (1/n_e) sum_a s(T_a), s = s0_e + s1_e T or the k table;
 * K0_e the element matrix at s = 1, symmetric), C_k = sum_e m_e c_e(T_k)
 * (c_e = c0_e + c1_e T or c0_e times the c table), m_e = rho_e V_e / n_e,
 * and Q_k = sum_f share_f [-h_f (T_k - Ta_f) - sigma eps_f ((T_k - Tz)^4 -
 * (Ta_f - Tz)^4) + q_f] + P_k.  Dirichlet nodes are reset to their values, so
 * their rows of the Jacobian vanish.  With lam = dL/dT', mu_k = dt_k lam_k / C_k
 * (0 on Dirichlet nodes) and dT = T' - T:
 *   dL/dT_j = lam_j (1 - dT_j C'_j / C_j)          C'_j = sum_{e owns j} m_e c_e'(T_j)
 *           - sum_{e owns j} [ s_e (K0_e mu_e)_j + s'(T_j) / n_e (mu_e . K0_e T_e) ]
 *           - mu_j sum_{f owns j} share_f (h_f + 4 sigma eps_f (T_j - Tz)^3),
 * set to 0 on Dirichlet nodes (their values are data, not state), and the
 * parameter derivatives accumulated over the steps are
 *   d/d log k_e (k_e scales K0_e):  -mu_e . F_e
 *   d/d c0_e:                       -m_e sum_{k of e, not Dirichlet} lam_k dT_k / C_k dc_e/dc0_e(T_k)
 *                                   (dc_e/dc0_e = 1, or the c table's value)
 *   d/d h_f:                        -share_f sum_{k of f} mu_k (T_k - Ta_f).
 * Runs the steps in reverse from hist (T^0..T^nsteps); on return lam holds
 * dL/dT^0.  is_dir[N] is 1 on Dirichlet nodes.  Returns 0, or -1 if a work
 * array could not be allocated.
 */
int orc_adjoint(const orc_problem *P, const double *hist, int64_t nsteps, const int8_t *is_dir,
                double *lam, double *g_logk, double *g_c, double *g_h) {
  const int ne = P->ne;
  const int64_t N = P->N, E = P->E;
  double *Fe = malloc(sizeof(double) * E * ne), *F = malloc(sizeof(double) * N);
  double *C = malloc(sizeof(double) * N), *Cp = calloc(N, sizeof(double));
  double *mu = malloc(sizeof(double) * N), *out = malloc(sizeof(double) * N);
  int rc = 0;
  if (!Fe || !F || !C || !Cp || !mu || !out) {
    rc = -1;
    goto done;
  }
  for (int64_t n = nsteps - 1; n >= 0; n--) {
    const double *Tn = hist + n * N, *Tn1 = hist + (n + 1) * N;
    orc_loads(P, Tn, Fe, F, C); /* F_e and C at T^n */
    memset(Cp, 0, sizeof(double) * N);
    for (int64_t e = 0; e < E; e++)
      for (int a = 0; a < ne; a++) {
        const int32_t k = P->conn[(int64_t)a * E + e];
        double dc;
        (void)cfun(P, e, Tn[k], &dc);
        Cp[k] += P->rho[e] * P->V[e] / ne * dc;
      }
    for (int64_t k = 0; k < N; k++) {
      mu[k] = is_dir[k] ? 0.0 : P->dt[k] * lam[k] / C[k];
      out[k] = is_dir[k] ? 0.0 : lam[k] * (1.0 - (Tn1[k] - Tn[k]) * Cp[k] / C[k]);
    }
    for (int64_t e = 0; e < E; e++) {
      double muF = 0, gc = 0, Kmu[8], Te[8], dse[8];
      int32_t kk[8];
      for (int a = 0; a < ne; a++) {
        kk[a] = P->conn[(int64_t)a * E + e];
        Te[a] = Tn[kk[a]];
      }
      const double se = kfac(P, e, Te, dse);
      element_apply(P, e, mu, se, Kmu); /* s_e K0_e mu_e */
      for (int a = 0; a < ne; a++) {
        muF += mu[kk[a]] * Fe[e * ne + a];
        /* dc_e/dc0_e at T_k: 1, or the c table's value */
        double sl, dcdc0 = 1.0;
        if (P->nct > 0) dcdc0 = table_eval(P->nct, P->ct_T, P->ct_f, Tn[kk[a]], &sl);
        if (!is_dir[kk[a]]) gc += lam[kk[a]] * (Tn1[kk[a]] - Tn[kk[a]]) / C[kk[a]] * dcdc0;
      }
      /* mu_e . K0_e T_e = mu_e . F_e / s_e, times d s_e / d T_a per node */
      const double muKT = muF / se;
      for (int a = 0; a < ne; a++) out[kk[a]] -= Kmu[a] + dse[a] * muKT;
      g_logk[e] += -muF;
      g_c[e] += -P->rho[e] * P->V[e] / ne * gc;
    }
    for (int64_t f = 0; f < P->nf; f++) {
      const double share = P->farea[f] / P->nfn;
      for (int b = 0; b < P->nfn; b++) {
        const int32_t k = P->faces[f * P->nfn + b];
        const double d = Tn[k] - P->Tz;
        out[k] -= mu[k] * share * (P->fh[f] + 4.0 * P->sigma * P->feps[f] * d * d * d);
        g_h[f] += -mu[k] * share * (Tn[k] - P->fTa[f]);
      }
    }
    for (int64_t k = 0; k < N; k++) lam[k] = is_dir[k] ? 0.0 : out[k];
  }
done:
  free(Fe);
  free(F);
  free(C);
  free(Cp);
  free(mu);
  free(out);
  return rc;
}
