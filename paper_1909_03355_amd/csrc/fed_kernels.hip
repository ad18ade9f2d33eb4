// HIP kernels of the FED-FEM library for gfx950 (MI355X).
//
// Pre-computation (Sec. 3.5 (i)) runs once in FP64.  The time step is one fused
// kernel per step: a workgroup owns a tile of nodes, stages their temperatures
// and those of the tile's halo in LDS, computes the loads of every element
// touching its nodes (Eq. 17-20), sums them per node in ascending element order
// through LDS slots (Eq. 10-11, no global K, no atomics), adds the surface loads
// (Eq. 4, 5, 7) and updates the node explicitly (Eq. 16).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>
#include <vector>

#include "fed_kernels.h"

namespace fed {

namespace {

constexpr double kSigma = 5.67e-8;  // Stefan-Boltzmann constant (Sec. 2)

__device__ __constant__ int8_t kHexS[8][3] = {
    {-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
    {-1, -1, 1},  {1, -1, 1},  {1, 1, 1},  {-1, 1, 1}};

inline int blocks_for(int64_t n, int bs) {
  int64_t b = (n + bs - 1) / bs;
  return (int)(b < 1 ? 1 : b);
}

// Largest eigenvalue of a symmetric 3x3 matrix by the cyclic Jacobi method
// (plane rotations that annihilate one off-diagonal entry at a time, as in
// Golub & Van Loan, Sec. 8.5).  Accurate to rounding also for repeated
// eigenvalues, where the closed-form cubic solution loses half the digits.
__device__ double sym3_lmax(double a00, double a11, double a22, double a01, double a12,
                            double a02) {
  double A[3][3] = {{a00, a01, a02}, {a01, a11, a12}, {a02, a12, a22}};
  for (int sweep = 0; sweep < 12; sweep++) {
    double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    if (off <= 1e-34 * dia) break;
    for (int p = 0; p < 2; p++)
      for (int q = p + 1; q < 3; q++) {
        double apq = A[p][q];
        if (apq == 0.0) continue;
        double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < 3; k++) {  // columns p, q
          double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - sn * akq;
          A[k][q] = sn * akp + c * akq;
        }
        for (int k = 0; k < 3; k++) {  // rows p, q
          double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - sn * aqk;
          A[q][k] = sn * apk + c * aqk;
        }
      }
  }
  double m = A[0][0];
  if (A[1][1] > m) m = A[1][1];
  if (A[2][2] > m) m = A[2][2];
  return m;
}

__device__ void inverse3(const double J[3][3], double d, double R[3][3]) {
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

__device__ double det3(const double J[3][3]) {
  return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
         J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
         J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

// ---------------------------------------------------------------------------
// Geometry (Sec. 3.2).  With B = J^{-T} dN/dxi at the integration point, the
// element load of Eq. 20 is F_e = W B^T D B T_e.  For the one-point hexahedron
// dN_a/dxi(0) = s_a / 8 (s_a the corner signs), so
//   F_a = s_a . Hhat (sum_b s_b T_b),  Hhat = W J^{-1} D J^{-T} / 64, W = 8 det J(0);
// for the linear tetrahedron, with d_i = T_i - T_0 and J = [x_i - x_0],
//   F_{1..3} = Hhat d,  F_0 = -(F_1 + F_2 + F_3),  Hhat = V J^{-1} D J^{-T}.
// Hhat (6 numbers, symmetric) is the precomputed "G D B" of Eq. 19-22.
// Natural signs (xi, eta, zeta) of the hexahedron's nodes in the local order
// of kHexS, and the hourglass patterns of Flanagan and Belytschko's orthogonal
// hourglass control (not in the paper): h_0 = eta zeta, h_1 = zeta xi,
// h_2 = xi eta, h_3 = xi eta zeta.
__host__ __device__ constexpr int hex_xi(int n) { return (n == 1 || n == 2 || n == 5 || n == 6) ? 1 : -1; }
__host__ __device__ constexpr int hex_eta(int n) { return (n >> 1 & 1) ? 1 : -1; }
__host__ __device__ constexpr int hex_zeta(int n) { return n >= 4 ? 1 : -1; }
__host__ __device__ constexpr int hg_sign(int al, int n) {
  return al == 0   ? hex_eta(n) * hex_zeta(n)
         : al == 1 ? hex_zeta(n) * hex_xi(n)
         : al == 2 ? hex_xi(n) * hex_eta(n)
                   : hex_xi(n) * hex_eta(n) * hex_zeta(n);
}
static_assert(hex_xi(0) == -1 && hex_xi(2) == 1 && hex_eta(3) == 1 && hex_eta(5) == -1 &&
                  hex_zeta(3) == -1 && hex_zeta(7) == 1,
              "node signs follow kHexS");

// Largest eigenvalue of a symmetric 8x8 matrix by the cyclic Jacobi method
// (rotations until the off-diagonal part is negligible; A is overwritten).
__device__ double sym8_lmax(double A[8][8]) {
  for (int sweep = 0; sweep < 50; sweep++) {
    double off = 0, diag = 0;
    for (int p = 0; p < 8; p++) {
      diag += A[p][p] * A[p][p];
      for (int q = p + 1; q < 8; q++) off += A[p][q] * A[p][q];
    }
    if (off <= 1e-32 * diag) break;
    for (int p = 0; p < 7; p++)
      for (int q = p + 1; q < 8; q++) {
        if (A[p][q] == 0.0) continue;
        const double th = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
        const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < 8; k++) {
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - sn * akq;
          A[k][q] = sn * akp + c * akq;
        }
        for (int k = 0; k < 8; k++) {
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - sn * aqk;
          A[q][k] = sn * apk + c * aqk;
        }
      }
  }
  double m = A[0][0];
  for (int p = 1; p < 8; p++) m = fmax(m, A[p][p]);
  return m;
}

__global__ void k_geom(GeomArgs a) {
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= a.E) return;
  const int ne = a.ne;
  double X[8][3];
  for (int n = 0; n < ne; n++) {
    int32_t k = a.conn[(int64_t)n * a.E + e];
    X[n][0] = a.x[k];
    X[n][1] = a.y[k];
    X[n][2] = a.z[k];
  }
  int m = a.emat ? a.emat[e] : 0;
  double dk[6];
  for (int r = 0; r < 6; r++) dk[r] = a.ek ? a.ek[(int64_t)r * a.E + e] : a.mats[m].k[r];
  double J[3][3], Ji[3][3], W, V, det;
  double M3[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // B B^T
  double bm[8][3];  // uniform-gradient hexahedron: the mean gradient of every shape function
  if (ne == 8) {
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) {
        double s = 0;
        for (int n = 0; n < 8; n++) s += X[n][i] * kHexS[n][j];
        J[i][j] = s / 8.0;
      }
    det = det3(J);
    W = 8.0 * det;
    // exact volume of the trilinear map: 2x2x2 Gauss points, unit weights
    const double g = 0.57735026918962576451;  // 1/sqrt(3), Gauss point of the 2-point rule
    V = 0;
    for (int qp = 0; qp < 8; qp++) {
      double p0 = kHexS[qp][0] * g, p1 = kHexS[qp][1] * g, p2 = kHexS[qp][2] * g;
      double Jq[3][3];
      for (int i = 0; i < 3; i++) {
        double s0 = 0, s1 = 0, s2 = 0;
        for (int n = 0; n < 8; n++) {
          double sx = kHexS[n][0], sy = kHexS[n][1], sz = kHexS[n][2];
          s0 += X[n][i] * sx * (1 + sy * p1) * (1 + sz * p2);
          s1 += X[n][i] * sy * (1 + sx * p0) * (1 + sz * p2);
          s2 += X[n][i] * sz * (1 + sx * p0) * (1 + sy * p1);
        }
        Jq[i][0] = s0 / 8.0;
        Jq[i][1] = s1 / 8.0;
        Jq[i][2] = s2 / 8.0;
      }
      V += det3(Jq);
    }
    if (!(det > 0.0)) {
      atomicAdd(a.nbad, 1);
      det = 1.0;
    }
    inverse3(J, det, Ji);
    if (a.hexmean) {
      // uniform gradient: mean of B over the element, 2x2x2 Gauss of B det J
      // (exact: a polynomial of degree <= 3 per natural coordinate), W = V
      double S[8][3] = {};
      for (int qp = 0; qp < 8; qp++) {
        double p0 = kHexS[qp][0] * g, p1 = kHexS[qp][1] * g, p2 = kHexS[qp][2] * g;
        double dN[8][3], Jq[3][3], Jqi[3][3];
        for (int n = 0; n < 8; n++) {
          double sx = kHexS[n][0], sy = kHexS[n][1], sz = kHexS[n][2];
          dN[n][0] = sx * (1 + sy * p1) * (1 + sz * p2) / 8.0;
          dN[n][1] = sy * (1 + sx * p0) * (1 + sz * p2) / 8.0;
          dN[n][2] = sz * (1 + sx * p0) * (1 + sy * p1) / 8.0;
        }
        for (int i = 0; i < 3; i++)
          for (int j = 0; j < 3; j++) {
            double t = 0;
            for (int n = 0; n < 8; n++) t += X[n][i] * dN[n][j];
            Jq[i][j] = t;
          }
        double dq = det3(Jq);
        if (!(dq > 0.0)) {
          atomicAdd(a.nbad, 1);
          dq = 1.0;
        }
        inverse3(Jq, dq, Jqi);
        for (int n = 0; n < 8; n++)
          for (int i = 0; i < 3; i++)
            S[n][i] += (Jqi[0][i] * dN[n][0] + Jqi[1][i] * dN[n][1] + Jqi[2][i] * dN[n][2]) * dq;
      }
      W = V;
      for (int n = 0; n < 8; n++) {
        double *b = bm[n];
        for (int i = 0; i < 3; i++) b[i] = S[n][i] / V;
        if (n < 7)
          for (int i = 0; i < 3; i++) a.H0[(int64_t)(3 * n + i) * a.E + e] = b[i];
        for (int i = 0; i < 3; i++)
          for (int j = 0; j < 3; j++) M3[i][j] += b[i] * b[j];
      }
    } else {
      // B B^T = J^{-T} (sum_a s_a s_a^T / 64) J^{-1}, formed from the columns of B
      for (int n = 0; n < 8; n++) {
        double b[3];
        for (int i = 0; i < 3; i++)
          b[i] = (Ji[0][i] * kHexS[n][0] + Ji[1][i] * kHexS[n][1] + Ji[2][i] * kHexS[n][2]) / 8.0;
        for (int i = 0; i < 3; i++)
          for (int j = 0; j < 3; j++) M3[i][j] += b[i] * b[j];
      }
    }
  } else {
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) J[i][j] = X[j + 1][i] - X[0][i];
    det = det3(J);
    V = fabs(det) / 6.0;
    W = V;
    if (det == 0.0) {
      atomicAdd(a.nbad, 1);
      det = 1.0;
    }
    inverse3(J, det, Ji);
    double b[4][3];
    for (int i = 0; i < 3; i++) {
      b[0][i] = 0;
      for (int n = 1; n < 4; n++) {
        b[n][i] = Ji[n - 1][i];  // grad N_n = J^{-T} e_{n-1}
        b[0][i] -= b[n][i];
      }
    }
    for (int n = 0; n < 4; n++)
      for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) M3[i][j] += b[n][i] * b[n][j];
  }
  // Hhat = c * Ji D Ji^T,  c = W/64 (hex) or V (tet)
  double D[3][3] = {{dk[0], dk[3], dk[5]}, {dk[3], dk[1], dk[4]}, {dk[5], dk[4], dk[2]}};
  double lam_hg = -1.0;  // set by the hourglass-controlled hexahedron
  double c = ne == 8 ? W / 64.0 : V;
  double T1[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++)
      T1[i][j] = Ji[i][0] * D[0][j] + Ji[i][1] * D[1][j] + Ji[i][2] * D[2][j];
  double Hm[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++)
      Hm[i][j] = c * (T1[i][0] * Ji[j][0] + T1[i][1] * Ji[j][1] + T1[i][2] * Ji[j][2]);
  if (ne == 8 && a.hexmean) {
    for (int r = 0; r < 6; r++) a.H0[(int64_t)(21 + r) * a.E + e] = V * dk[r];
    if (a.hg_eps > 0) {
      // hourglass control: kappa = eps (tr D / 3) V sum_a |b_a|^2 (row 27, takes
      // the per-element factor) and h_alpha . x_i (rows 28 + 3 alpha + i)
      double bb = 0;
      for (int n = 0; n < 8; n++) bb += bm[n][0] * bm[n][0] + bm[n][1] * bm[n][1] + bm[n][2] * bm[n][2];
      const double kap = a.hg_eps * (dk[0] + dk[1] + dk[2]) / 3.0 * V * bb;
      a.H0[(int64_t)27 * a.E + e] = kap;
      double gam[4][8];
      for (int al = 0; al < 4; al++) {
        double hx[3] = {0, 0, 0};
        for (int n = 0; n < 8; n++)
          for (int i = 0; i < 3; i++) hx[i] += hg_sign(al, n) * X[n][i];
        for (int i = 0; i < 3; i++) a.H0[(int64_t)(28 + 3 * al + i) * a.E + e] = hx[i];
        for (int n = 0; n < 8; n++)
          gam[al][n] = (hg_sign(al, n) - (hx[0] * bm[n][0] + hx[1] * bm[n][1] + hx[2] * bm[n][2])) / 8.0;
      }
      // stability: lambda_max of the whole element matrix V b D b^T + kappa G^T G
      double K8[8][8];
      for (int p = 0; p < 8; p++)
        for (int q = 0; q < 8; q++) {
          double t = 0;
          for (int i = 0; i < 3; i++)
            for (int j = 0; j < 3; j++) t += bm[p][i] * D[i][j] * bm[q][j];
          double g2 = 0;
          for (int al = 0; al < 4; al++) g2 += gam[al][p] * gam[al][q];
          K8[p][q] = V * t + kap * g2;
        }
      lam_hg = sym8_lmax(K8) / V;
    }
  } else {
    a.H0[0 * a.E + e] = Hm[0][0];
    a.H0[1 * a.E + e] = Hm[1][1];
    a.H0[2 * a.E + e] = Hm[2][2];
    a.H0[3 * a.E + e] = 0.5 * (Hm[0][1] + Hm[1][0]);
    a.H0[4 * a.E + e] = 0.5 * (Hm[1][2] + Hm[2][1]);
    a.H0[5 * a.E + e] = 0.5 * (Hm[0][2] + Hm[2][0]);
  }
  a.V[e] = V;
  // stability: lambda_max(K_e) = W lambda_max(L^T B B^T L) with D = L L^T (Cholesky)
  double l00 = dk[0];
  bool spd = l00 > 0;
  l00 = spd ? sqrt(l00) : 1.0;
  double l10 = dk[3] / l00, l20 = dk[5] / l00;
  double t11 = dk[1] - l10 * l10;
  spd = spd && t11 > 0;
  double l11 = t11 > 0 ? sqrt(t11) : 1.0;
  double l21 = (dk[4] - l20 * l10) / l11;
  double t22 = dk[2] - l20 * l20 - l21 * l21;
  spd = spd && t22 > 0;
  double l22 = t22 > 0 ? sqrt(t22) : 1.0;
  if (!spd) atomicAdd(a.nnotspd, 1);
  double L[3][3] = {{l00, 0, 0}, {l10, l11, 0}, {l20, l21, l22}};
  double ML[3][3], A[3][3];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++)
      ML[i][j] = M3[i][0] * L[0][j] + M3[i][1] * L[1][j] + M3[i][2] * L[2][j];
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) A[i][j] = L[0][i] * ML[0][j] + L[1][i] * ML[1][j] + L[2][i] * ML[2][j];
  double lm = sym3_lmax(A[0][0], A[1][1], A[2][2], 0.5 * (A[0][1] + A[1][0]),
                        0.5 * (A[1][2] + A[2][1]), 0.5 * (A[0][2] + A[2][0]));
  a.lamgeo[e] = lam_hg >= 0 ? lam_hg : (V > 0 ? W / V : 0.0) * lm;
}

// Lumped (diagonal) heat capacity (Sec. 3.1, Eq. 13-14): every element gives
// rho V / n_e to each of its nodes; C_k(T) = M0_k + M1_k T.  Summed in
// ascending element order per node.
__global__ void k_mass(MassArgs a) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= a.N) return;
  double m0 = 0, m1 = 0, cm = 0;
  for (int64_t p = a.inc_ptr[k]; p < a.inc_ptr[k + 1]; p++) {
    int32_t e = a.inc_elem[p];
    const MatDev &mt = a.mats[a.emat ? a.emat[e] : 0];
    double v = mt.rho * a.V[e] / a.ne;
    const double c0 = a.ec0 ? a.ec0[e] : mt.c0;
    double clo = c0 + mt.c1 * a.T_lo, chi = c0 + mt.c1 * a.T_hi;
    m0 += v * c0;
    m1 += v * mt.c1;
    cm += v * (clo < chi ? clo : chi) * a.fc_min;
  }
  a.M0[k] = m0;
  a.M1[k] = m1;
  a.Cmin[k] = cm;
}

// Face areas: triangles by the cross product, bilinear quadrilaterals by a
// 2x2 Gauss rule on |x_u x x_v|.
__global__ void k_face_area(BndArgs a) {
  int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f >= a.nf) return;
  double X[4][3];
  for (int b = 0; b < a.nfn; b++) {
    int32_t k = a.faces[f * a.nfn + b];
    X[b][0] = a.x[k];
    X[b][1] = a.y[k];
    X[b][2] = a.z[k];
  }
  double area = 0;
  if (a.nfn == 3) {
    double u[3], v[3];
    for (int i = 0; i < 3; i++) {
      u[i] = X[1][i] - X[0][i];
      v[i] = X[2][i] - X[0][i];
    }
    double c0 = u[1] * v[2] - u[2] * v[1], c1 = u[2] * v[0] - u[0] * v[2],
           c2 = u[0] * v[1] - u[1] * v[0];
    area = 0.5 * sqrt(c0 * c0 + c1 * c1 + c2 * c2);
  } else {
    const double g = 0.57735026918962576451;
    const double su[4] = {-1, 1, 1, -1}, sv[4] = {-1, -1, 1, 1};
    for (int qp = 0; qp < 4; qp++) {
      double pu = su[qp] * g, pv = sv[qp] * g;
      double xu[3] = {0, 0, 0}, xv[3] = {0, 0, 0};
      for (int b = 0; b < 4; b++) {
        double du = su[b] * (1 + sv[b] * pv) * 0.25, dv = sv[b] * (1 + su[b] * pu) * 0.25;
        for (int i = 0; i < 3; i++) {
          xu[i] += X[b][i] * du;
          xv[i] += X[b][i] * dv;
        }
      }
      double c0 = xu[1] * xv[2] - xu[2] * xv[1], c1 = xu[2] * xv[0] - xu[0] * xv[2],
             c2 = xu[0] * xv[1] - xu[1] * xv[0];
      area += sqrt(c0 * c0 + c1 * c1 + c2 * c2);
    }
  }
  a.farea[f] = area;
}

// Applied power of boundary record r: flux q A of its faces (|f| / n_f each)
// plus the concentrated loads W of its point items, in item order.  Shared by
// the record refresh and the per-step rows of a point-load schedule, so a row
// equals the record a refresh with the same loads derives, bit for bit.
__device__ inline double rec_power(const BndArgs &a, int64_t r, const double *W) {
#pragma clang fp contract(off)
  double P = 0;
  for (int64_t p = a.rec_ptr[r]; p < a.rec_ptr[r + 1]; p++) {
    const int32_t it = a.rec_item[p];
    if (it >= 0) {
      const double s = a.farea[it] / a.nfn, q = a.fq ? a.fq[it] : 0.0;
      P += q * s;
    } else {
      P += W[-(it + 1)];
    }
  }
  return P;
}

// Per boundary node: lumped convection h A, h A Ta, radiation sigma eps A and the
// applied power (flux q A plus concentrated loads), each face giving |f| / n_f.
__global__ void k_bnd_rec(BndArgs a) {
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= a.nrec) return;
  double hA = 0, hAT = 0, eA = 0, rTa = 0;
  bool rad = false;
  for (int64_t p = a.rec_ptr[r]; p < a.rec_ptr[r + 1]; p++) {
    int32_t it = a.rec_item[p];
    if (it >= 0) {
      double s = a.farea[it] / a.nfn;
      double h = a.fh ? a.fh[it] : 0.0, Ta = a.fTa ? a.fTa[it] : 0.0;
      double eps = a.feps ? a.feps[it] : 0.0;
      hA += h * s;
      hAT += h * s * Ta;
      eA += kSigma * eps * s;
      if (eps > 0 && !rad) {
        rad = true;
        rTa = Ta;
      }
    }
  }
  a.bhA[r] = hA;
  a.bhAT[r] = hAT;
  a.beA[r] = eA;
  a.bP[r] = rec_power(a, r, a.pt_W);
  if (a.bTa) a.bTa[r] = rTa;
}

// Rows of a point-load schedule: out[row][r] = (R) rec_power(r, W[row])
template <typename R>
__global__ void k_point_rows(BndArgs a, int64_t nrows, int64_t npt, const double *W, R *out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nrows * a.nrec) return;
  const int64_t row = i / a.nrec, r = i - row * a.nrec;
  out[i] = (R)rec_power(a, r, W + row * npt);
}

// Stability bound (Sec. 3.4): per element lambda_e = lambda_max(K_e(T)) / (rho c V /
// n_e) at the largest D and smallest c over [T_lo, T_hi]; per boundary node the
// convection and linearised radiation rate; maxima per instance.
__global__ void k_dt_elem(DtArgs a) {
  // one atomic per run of equal instances in a wave: elements of an instance
  // are contiguous, so a wave-wide max for the wave's first instance plus
  // per-thread atomics for the rest keeps contention low
  __shared__ double smax[1024 / 64];
  int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double lam = 0;
  int inst = -1;
  if (e < a.E) {
    const MatDev &mt = a.mats[a.emat ? a.emat[e] : 0];
    double slo = mt.s0 + mt.s1 * a.T_lo, shi = mt.s0 + mt.s1 * a.T_hi;
    const double c0 = a.ec0 ? a.ec0[e] : mt.c0;
    double clo = c0 + mt.c1 * a.T_lo, chi = c0 + mt.c1 * a.T_hi;
    double smax_ = (slo > shi ? slo : shi) * a.fk_max, cmin = (clo < chi ? clo : chi) * a.fc_min;
    double ks = a.kscale ? a.kscale[e] : 1.0;
    lam = a.ne * ks * smax_ * a.lamgeo[e] / (mt.rho * cmin);
    inst = a.elem_inst ? a.elem_inst[e] : 0;
  }
  int64_t e0 = blockIdx.x * (int64_t)blockDim.x;
  int inst0 = a.elem_inst ? a.elem_inst[e0] : 0;
  bool same = inst == inst0;
  double v = same ? lam : 0.0;
  for (int off = 32; off > 0; off >>= 1) {
    double o = __shfl_down(v, off, 64);
    v = o > v ? o : v;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) smax[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); i++) m = smax[i] > m ? smax[i] : m;
    if (m > 0) atomicMax(&a.lamE[inst0], (unsigned long long)__double_as_longlong(m));
  }
  if (!same && inst >= 0 && lam > 0)
    atomicMax(&a.lamE[inst], (unsigned long long)__double_as_longlong(lam));
}

__global__ void k_dt_node(DtArgs a) {
  // boundary records of an instance are contiguous (tiles never mix instances):
  // a block-wide max for the block's first instance plus per-thread atomics for
  // the others keeps contention low
  __shared__ double smax[1024 / 64];
  int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double lam = 0;
  int inst = -1;
  if (r < a.nrec) {
    int32_t k = a.rec_node[r];
    double d = a.T_hi - a.Tz;
    lam = (a.bhA[r] + 4.0 * a.beA[r] * d * d * d) / a.Cmin[k];
    inst = a.node_inst ? a.node_inst[k] : 0;
  }
  const int64_t r0 = blockIdx.x * (int64_t)blockDim.x;
  const int inst0 = a.node_inst ? a.node_inst[a.rec_node[r0]] : 0;
  const bool same = inst == inst0;
  double v = same ? lam : 0.0;
  for (int off = 32; off > 0; off >>= 1) {
    double o = __shfl_down(v, off, 64);
    v = o > v ? o : v;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) smax[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); i++) m = smax[i] > m ? smax[i] : m;
    if (m > 0) atomicMax(&a.lamB[inst0], (unsigned long long)__double_as_longlong(m));
  }
  if (!same && inst >= 0 && lam > 0)
    atomicMax(&a.lamB[inst], (unsigned long long)__double_as_longlong(lam));
}

// Working arrays of the step in precision R: per node alpha = M0 / dt and
// beta = M1 / dt (the inverse of A / c(T) of Eq. 15-16: dT = (Q - F) / (alpha +
// beta T)); alpha = +inf holds a Dirichlet node fixed.  Boundary records and the
// expanded element operators are cast to R.
template <typename R>
__global__ void k_node_arrays(NodeArrArgs a) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  R *alpha = (R *)a.alpha, *beta = (R *)a.beta;
  if (i < a.N) {
    double dt = a.dt_inst[a.node_inst ? a.node_inst[i] : 0];
    if (a.is_dir[i]) {
      alpha[i] = (R)INFINITY;
      beta[i] = 0;
    } else {
      alpha[i] = (R)(a.M0[i] / dt);
      beta[i] = (R)(a.M1[i] / dt);
    }
  }
  if (i < a.nrec) {
    ((R *)a.rA)[i] = (R)a.bhA[i];
    ((R *)a.rAT)[i] = (R)a.bhAT[i];
    ((R *)a.reA)[i] = (R)a.beA[i];
    ((R *)a.rTa)[i] = (R)a.bTa[i];
    ((R *)a.rP)[i] = (R)a.bP[i];
  }
}

template <typename R>
__global__ void k_expand_sk(int64_t Eexp, const int32_t *eorig, const MatDev *mats,
                            const int32_t *emat, R *esk) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= Eexp) return;
  const MatDev &mt = mats[emat ? emat[eorig[i]] : 0];
  esk[i] = (R)mt.s0;
  esk[Eexp + i] = (R)mt.s1;
}

template <typename R>
__global__ void k_expand_H(int W, int from, int to, int64_t Eexp, int64_t E, const int32_t *eorig,
                           const double *H0, const double *kscale, R *H) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= Eexp) return;
  int32_t e = eorig[i];
  double ks = kscale ? kscale[e] : 1.0;
  for (int r = 0; r < W; r++)
    H[(int64_t)r * Eexp + i] =
        (R)(r >= from && r < to ? H0[(int64_t)r * E + e] * ks : H0[(int64_t)r * E + e]);
}

// ---------------------------------------------------------------------------
// The step.  One workgroup per tile; the XCD-aware block->tile map keeps a run of
// spatially adjacent tiles on one XCD (blocks are dealt to the 8 XCDs round
// robin), so halo re-reads and the next step's re-reads of the same tiles hit
// that XCD's L2.
// Piecewise-linear table of n breakpoints T_i (increasing) followed by n
// values, constant beyond its ends; slope receives the derivative (0 beyond
// the ends, the left segment's at a breakpoint).
template <typename R>
__device__ inline R table_eval(const R *tab, int n, R T, R &slope) {
#pragma clang fp contract(off)
  if (!(T > tab[0])) {
    slope = (R)0;
    return tab[n];
  }
  if (!(T < tab[n - 1])) {
    slope = (R)0;
    return tab[2 * n - 1];
  }
  int i = 1;
  while (T > tab[i]) i++;
  const R h = tab[i] - tab[i - 1], df = tab[n + i] - tab[n + i - 1];
  slope = df / h;
  return fma((T - tab[i - 1]) / h, df, tab[n + i - 1]);
}

// pairwise sums of an element's nodal values, in the order every kernel uses
template <typename R, int NE>
__device__ inline R node_sum(const R *v) {
#pragma clang fp contract(off)
  if constexpr (NE == 8) return ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
  else return (v[0] + v[1]) + (v[2] + v[3]);
}

// Conductivity factor s_e of an element (Sec. 4.2.2): the property is
// evaluated at each node of the element from that node's temperature and the
// nodal values are averaged for the element.  For the linear law s0 + s1 T
// that average is s0 + s1 Tbar, which is how it is evaluated; the shared
// multiplier table (n > 0) is evaluated at every node.  slope(T_a) is
// n_e d s_e / d T_a, the law's slope at node a.
template <typename R>
struct KLaw {
  R s0, s1;
  const R *tab;
  int n;
  // table laws in the forward kernels: the table's value at every touched node
  // of the tile, evaluated once per node and step where its temperature is
  // staged (LDS, indexed like the temperatures); null: evaluated per element
  R *nv = nullptr;
  // the element mean of its nodes' table values V (the same sums as elem)
  template <int NE>
  __device__ R mean(const R *V) const {
#pragma clang fp contract(off)
    R f = V[0];
#pragma unroll
    for (int a = 1; a < NE; a++) f = f + V[a];
    return f * ((R)1 / (R)NE);
  }
  // s_e of an element whose nodes sit at local indices loc
  template <int NE>
  __device__ R elem_at(const R *T, const uint32_t *loc) const {
    if (n && nv) {
      R V[NE];
#pragma unroll
      for (int a = 0; a < NE; a++) V[a] = nv[loc[a]];
      return mean<NE>(V);
    }
    return elem<NE>(T);
  }
  // the table's value at one node, staged into nv[j]
  __device__ void stage(int j, R T) const {
    R sl;
    nv[j] = table_eval(tab, n, T, sl);
  }
  template <int NE>
  __device__ R elem(const R *T) const {
#pragma clang fp contract(off)
    if (n) {
      // summed node by node (one value live at a time)
      R sl, f = table_eval(tab, n, T[0], sl);
#pragma unroll
      for (int a = 1; a < NE; a++) f = f + table_eval(tab, n, T[a], sl);
      return f * ((R)1 / (R)NE);
    }
    return fma(s1, node_sum<R, NE>(T) * ((R)1 / (R)NE), s0);
  }
  // the law's slope at one node temperature
  __device__ R slope(R T) const {
    if (n) {
      R sl;
      (void)table_eval(tab, n, T, sl);
      return sl;
    }
    return s1;
  }
};

template <typename R, int NE>
struct Elem;

template <typename R>
struct Elem<R, 8> {
  // F_a = s_a . (s * Hhat u),  u = sum_b s_b T_b written as sums of edge
  // differences (each a difference of nearby values, so exact or nearly so).
  __device__ static void load(const R *Tl, const uint32_t *loc, const KLaw<R> &kl, bool tdk,
                              const R h[6], R F[8]) {
    R T[8];
#pragma unroll
    for (int n = 0; n < 8; n++) T[n] = Tl[loc[n]];
    const bool staged = kl.n && kl.nv;
    R V[8];
    if (staged)
#pragma unroll
      for (int n = 0; n < 8; n++) V[n] = kl.nv[loc[n]];
    load_vals(T, V, staged, kl, tdk, h, F);
  }
  // V: the nodes' staged table values when staged
  __device__ static void load_vals(const R *T, const R *V, bool staged, const KLaw<R> &kl,
                                   bool tdk, const R h[6], R F[8]) {
    // rounding fixed by the source in every kernel that inlines this (no
    // FMA contraction; the FMAs are written out), so all step kernels agree
    // bit for bit
    #pragma clang fp contract(off)
    const R T0 = T[0], T1 = T[1], T2 = T[2], T3 = T[3], T4 = T[4], T5 = T[5], T6 = T[6], T7 = T[7];
    R ux = ((T1 - T0) + (T2 - T3)) + ((T5 - T4) + (T6 - T7));
    R uy = ((T3 - T0) + (T2 - T1)) + ((T7 - T4) + (T6 - T5));
    R uz = ((T4 - T0) + (T5 - T1)) + ((T6 - T2) + (T7 - T3));
    R s = kl.s0;
    if (tdk) s = staged ? kl.template mean<8>(V) : kl.template elem<8>(T);
    apply(s, h, ux, uy, uz, F);
  }
  // F from the gradient sums u and the factor s
  __device__ static void apply(R s, const R h[6], R ux, R uy, R uz, R F[8]) {
    #pragma clang fp contract(off)
    R qx = s * fma(h[5], uz, fma(h[3], uy, h[0] * ux));
    R qy = s * fma(h[4], uz, fma(h[1], uy, h[3] * ux));
    R qz = s * fma(h[2], uz, fma(h[4], uy, h[5] * ux));
    R a = qx + qy, b = qx - qy;
    F[0] = -a - qz;
    F[1] = b - qz;
    F[2] = a - qz;
    F[3] = -b - qz;
    F[4] = -a + qz;
    F[5] = b + qz;
    F[6] = a + qz;
    F[7] = -b + qz;
  }
};

template <typename R>
struct Elem<R, 4> {
  __device__ static void load(const R *Tl, const uint32_t *loc, const KLaw<R> &kl, bool tdk,
                              const R h[6], R F[4]) {
    #pragma clang fp contract(off)
    const R T[4] = {Tl[loc[0]], Tl[loc[1]], Tl[loc[2]], Tl[loc[3]]};
    R d1 = T[1] - T[0], d2 = T[2] - T[0], d3 = T[3] - T[0];
    R s = kl.s0;
    if (tdk) s = kl.template elem_at<4>(T, loc);
    apply(s, h, d1, d2, d3, F);
  }
  __device__ static void apply(R s, const R h[6], R d1, R d2, R d3, R F[4]) {
    #pragma clang fp contract(off)
    F[1] = s * fma(h[5], d3, fma(h[3], d2, h[0] * d1));
    F[2] = s * fma(h[4], d3, fma(h[1], d2, h[3] * d1));
    F[3] = s * fma(h[2], d3, fma(h[4], d2, h[5] * d1));
    F[0] = -((F[1] + F[2]) + F[3]);
  }
};

// Uniform-gradient (element-mean) hexahedron: F_a = b_a . q with
// q = s (V D) g and g = sum_b b_b T_b, where b_a are the columns of the mean
// gradient operator (b_7 = -(b_0 + ... + b_6), so g = sum_{a<7} b_a (T_a - T_7)).
// hb holds b_0..b_6 (21 values, b_a at 3a..3a+2) and V D (xx, yy, zz, xy, yz,
// xz) with the per-element conductivity factor folded in.
template <typename R>
struct ElemMean {
  __device__ static void load(const R *Tl, const uint32_t *loc, const KLaw<R> &kl, bool tdk,
                              const R hb[27], R F[8]) {
    #pragma clang fp contract(off)
    R T[8];
#pragma unroll
    for (int n = 0; n < 8; n++) T[n] = Tl[loc[n]];
    // (the FMAs written out, as in Elem<R, 8>, so every kernel rounds alike)
    R d = T[0] - T[7];
    R gx = hb[0] * d, gy = hb[1] * d, gz = hb[2] * d;
#pragma unroll
    for (int n = 1; n < 7; n++) {
      d = T[n] - T[7];
      gx = fma(hb[3 * n], d, gx);
      gy = fma(hb[3 * n + 1], d, gy);
      gz = fma(hb[3 * n + 2], d, gz);
    }
    R s = kl.s0;
    if (tdk) s = kl.template elem_at<8>(T, loc);
    const R *vd = hb + 21;
    const R qx = s * fma(vd[5], gz, fma(vd[3], gy, vd[0] * gx));
    const R qy = s * fma(vd[4], gz, fma(vd[1], gy, vd[3] * gx));
    const R qz = s * fma(vd[2], gz, fma(vd[4], gy, vd[5] * gx));
    R sum = 0;
#pragma unroll
    for (int n = 0; n < 7; n++) {
      F[n] = fma(hb[3 * n + 2], qz, fma(hb[3 * n + 1], qy, hb[3 * n] * qx));
      sum += F[n];
    }
    F[7] = -sum;
  }
};

// Uniform-gradient hexahedron with hourglass control (not in the paper: the
// scalar-field form of Flanagan and Belytschko's orthogonal hourglass
// control).  The load of ElemMean plus s kappa sum_alpha c_alpha gamma_alpha,
// where gamma_alpha,n = (h_alpha,n - hx_alpha . b_n) / 8 vanishes on linear
// fields and c_alpha = gamma_alpha . T = (h_alpha . T - hx_alpha . g) / 8.
// hb as for ElemMean, then hb[27] = kappa (with the per-element factor) and
// hb[28 + 3 alpha + i] = hx_alpha,i = h_alpha . x_i.
template <typename R>
struct ElemMeanHg {
  // hourglass amplitudes c_alpha from the differences d_n = T_n - T_7 (the
  // patterns sum to zero) and the mean gradient g
  __device__ static void amps(const R d[7], R gx, R gy, R gz, const R *hb, R c[4]) {
    #pragma clang fp contract(off)
#pragma unroll
    for (int al = 0; al < 4; al++) {
      R ht = 0;
#pragma unroll
      for (int n = 0; n < 7; n++) ht = hg_sign(al, n) > 0 ? ht + d[n] : ht - d[n];
      const R *hx = hb + 28 + 3 * al;
      c[al] = (ht - fma(hx[2], gz, fma(hx[1], gy, hx[0] * gx))) * (R)0.125;
    }
  }
  __device__ static void load(const R *Tl, const uint32_t *loc, const KLaw<R> &kl, bool tdk,
                              const R hb[40], R F[8]) {
    #pragma clang fp contract(off)
    R T[8], d[7];
#pragma unroll
    for (int n = 0; n < 8; n++) T[n] = Tl[loc[n]];
    d[0] = T[0] - T[7];
    R gx = hb[0] * d[0], gy = hb[1] * d[0], gz = hb[2] * d[0];
#pragma unroll
    for (int n = 1; n < 7; n++) {
      d[n] = T[n] - T[7];
      gx = fma(hb[3 * n], d[n], gx);
      gy = fma(hb[3 * n + 1], d[n], gy);
      gz = fma(hb[3 * n + 2], d[n], gz);
    }
    R s = kl.s0;
    if (tdk) s = kl.template elem_at<8>(T, loc);
    const R *vd = hb + 21;
    const R qx = s * fma(vd[5], gz, fma(vd[3], gy, vd[0] * gx));
    const R qy = s * fma(vd[4], gz, fma(vd[1], gy, vd[3] * gx));
    const R qz = s * fma(vd[2], gz, fma(vd[4], gy, vd[5] * gx));
    R c[4];
    amps(d, gx, gy, gz, hb, c);
    R w0 = c[0] * hb[28], w1 = c[0] * hb[29], w2 = c[0] * hb[30];
#pragma unroll
    for (int al = 1; al < 4; al++) {
      w0 = fma(c[al], hb[28 + 3 * al], w0);
      w1 = fma(c[al], hb[29 + 3 * al], w1);
      w2 = fma(c[al], hb[30 + 3 * al], w2);
    }
    const R sk = s * hb[27] * (R)0.125;
    R sum = 0;
#pragma unroll
    for (int n = 0; n < 7; n++) {
      R hc = 0;
#pragma unroll
      for (int al = 0; al < 4; al++) hc = hg_sign(al, n) > 0 ? hc + c[al] : hc - c[al];
      const R wb = fma(w2, hb[3 * n + 2], fma(w1, hb[3 * n + 1], w0 * hb[3 * n]));
      F[n] = fma(sk, hc - wb, fma(hb[3 * n + 2], qz, fma(hb[3 * n + 1], qy, hb[3 * n] * qx)));
      sum += F[n];
    }
    F[7] = -sum;
  }
};

// element operator by kind: OP 0 the folded 3x3 operator of Eq. 17-22 (6
// values), OP 1 the uniform-gradient hexahedron (27 values), OP 2 the same with
// hourglass control (40 values)
template <typename R, int NE, int OP>
struct Op {
  static constexpr int W = 6;
  __device__ static void load(const R *Tl, const uint32_t *loc, const KLaw<R> &kl, bool tdk,
                              const R *h, R *F) {
    Elem<R, NE>::load(Tl, loc, kl, tdk, h, F);
  }
};
template <typename R>
struct Op<R, 8, 1> {
  static constexpr int W = 27;
  __device__ static void load(const R *Tl, const uint32_t *loc, const KLaw<R> &kl, bool tdk,
                              const R *h, R *F) {
    ElemMean<R>::load(Tl, loc, kl, tdk, h, F);
  }
};
template <typename R>
struct Op<R, 8, 2> {
  static constexpr int W = 40;
  __device__ static void load(const R *Tl, const uint32_t *loc, const KLaw<R> &kl, bool tdk,
                              const R *h, R *F) {
    ElemMeanHg<R>::load(Tl, loc, kl, tdk, h, F);
  }
};

// packed per-element entries: 8 x u16 (hexahedra) or 4 x u16 (tetrahedra)
template <int NE>
struct Ent;
template <>
struct Ent<8> {
  using T = uint4;
  __device__ static void unpack(const uint4 &w, uint32_t v[8]) {
    v[0] = w.x & 0xffff; v[1] = w.x >> 16; v[2] = w.y & 0xffff; v[3] = w.y >> 16;
    v[4] = w.z & 0xffff; v[5] = w.z >> 16; v[6] = w.w & 0xffff; v[7] = w.w >> 16;
  }
};
template <>
struct Ent<4> {
  using T = uint2;
  __device__ static void unpack(const uint2 &w, uint32_t v[4]) {
    v[0] = w.x & 0xffff; v[1] = w.x >> 16; v[2] = w.y & 0xffff; v[3] = w.y >> 16;
  }
};

// Streamed element data read once per one-step launch: non-temporal loads,
// so it does not displace from the caches the data that launch reads again
// (halo temperatures, neighbouring tiles' nodes).  Measured on the two large
// streaming workloads: the operators' loads so marked cut the step 12%
// (tetrahedra) and 7% (hexahedra); the packed entries so marked help the
// hexahedra (another 8%) but cost the tetrahedra 14%, so ld_entries marks
// only the hexahedra's; marking also the node coefficients and the stores of
// the new state costs up to 15%.
template <typename R>
__device__ inline R ld_stream(const R *p) {
  return __builtin_nontemporal_load(p);
}
__device__ inline uint4 ld_stream(const uint4 *p) {
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
  return make_uint4(v.x, v.y, v.z, v.w);
}
// packed entries: non-temporal for hexahedra (above), plain for tetrahedra
__device__ inline uint4 ld_entries(const uint4 *p) { return ld_stream(p); }
__device__ inline uint2 ld_entries(const uint2 *p) { return *p; }

// element loads of one expanded element into the LDS slots of the nodes that
// this sub-step updates (local index < nupd); slot (node j, position p) lives at
// p * stride + j
// NM: node-major slots, every touched node's (node j, position p) at
// j * (2^pb + 1) + p, which is the packed entry plus the local index: no
// multiply, no test (the halo nodes' slots take the values no owned node
// needs), and an odd stride keeps the LDS banks of neighbouring nodes apart.
template <typename R, int NE, bool TDK, int OP = 0, bool NM = false>
__device__ inline void element_to_slots(const typename Ent<NE>::T &w, const R *h, const R *Tl,
                                        R *slot, int stride, int nupd, int pb, uint32_t pmask,
                                        const KLaw<R> &kl) {
  uint32_t v[NE], loc[NE];
  Ent<NE>::unpack(w, v);
#pragma unroll
  for (int n = 0; n < NE; n++) loc[n] = v[n] >> pb;
  R F[NE];
  Op<R, NE, OP>::load(Tl, loc, kl, TDK, h, F);
#pragma unroll
  for (int n = 0; n < NE; n++)
    if (NM) slot[v[n] + loc[n]] = F[n];
    else if (loc[n] < (uint32_t)nupd) slot[(v[n] & pmask) * stride + loc[n]] = F[n];
}

// law of expanded element e: the shared one, or the element's material's
// (s0, s1) when the materials differ in their k(T)
template <bool GEN, typename R, typename Args>
__device__ inline KLaw<R> elem_law(const Args &a, const KLaw<R> &kl, int64_t e) {
  KLaw<R> k = kl;
  if (GEN && a.esk) {
    k.s0 = ((const R *)a.esk)[e];
    k.s1 = ((const R *)a.esk)[a.Eexp + e];
  }
  return k;
}

// GEN: the kernel instance for tables and per-element laws; the others compile
// the shared linear law only
template <typename R, bool GEN>
__device__ inline KLaw<R> step_law(const StepArgs &a) {
  if (GEN) return KLaw<R>{(R)a.s0, (R)a.s1, (const R *)a.ktab, a.nkt};
  return KLaw<R>{(R)a.s0, (R)a.s1, nullptr, 0};
}

// capacity denominator alpha + beta T, or alpha times the shared c table
template <typename R>
__device__ inline R cap_den(R alpha, R beta, R T, const R *ctab, int nct) {
#pragma clang fp contract(off)
  if (nct) {
    R sl;
    return alpha * table_eval(ctab, nct, T, sl);
  }
  return fma(beta, T, alpha);
}

// ---- in-run health check ----------------------------------------------------
// (a temperature outside [win_lo, win_hi], the range the stability bound of
// Sec. 3.4 was derived for widened by the caller's margin, or not finite)
template <typename R>
__device__ inline bool outside(R T, R lo, R hi) {
  return !(T >= lo && T <= hi);
}

// the window in the working precision (kernel arguments: scalar registers)
template <typename R>
__device__ inline R win_lo(const StepArgs &a) {
  if constexpr (sizeof(R) == 4) return a.win_lo_f;
  else return a.win_lo;
}
template <typename R>
__device__ inline R win_hi(const StepArgs &a) {
  if constexpr (sizeof(R) == 4) return a.win_hi_f;
  else return a.win_hi;
}

// the launch's step count before its first step (graph replays add the base
// the replay started from)
__device__ inline long long health_step0(const StepArgs &a) {
  return a.step0 + (a.hbase ? __hip_atomic_load(&a.hl->base, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT)
                            : 0LL);
}

// records that a temperature left the window after step count n
__device__ inline void health_bad(const StepArgs &a, long long n) {
  __hip_atomic_fetch_min(&a.hl->first_bad, (unsigned long long)n, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
}

// Energy balance of one owned node after its update (summed over all nodes it
// is zero: the explicit update gives den dT = Q - F at every node that is not
// Dirichlet, and the conductive loads F of every element sum to zero, so
// sum_{not Dirichlet} (den dT - Q) - sum_{Dirichlet} F = -sum_k F_k = 0).  r
// collects the terms, s their magnitudes and |F|.
template <typename R, int MODE>
__device__ inline void energy_terms(R den, R Q, R F, R hi0, float lo0, R hi1, float lo1,
                                    double &r, double &s) {
  const double f = (double)F;
  if (!(den < (R)INFINITY)) {  // Dirichlet: den = +inf, T held
    r -= f;
    s += fabs(f);
    return;
  }
  double dT = (double)hi1 - (double)hi0;
  if (MODE == 1) dT += (double)lo1 - (double)lo0;
  const double e = (double)den * dT, q = (double)Q;
  r += e - q;
  s += (fabs(e) + fabs(q)) + fabs(f);
}

// Sum of (r, s) over the block in a fixed order, valid in thread 0 (every
// thread of the block calls it).
__device__ inline void block_sum2(double &r, double &s, double *red) {
  for (int o = 32; o > 0; o >>= 1) {
    r += __shfl_xor(r, o, 64);
    s += __shfl_xor(s, o, 64);
  }
  const int w = threadIdx.x >> 6, nw = (int)(blockDim.x + 63) >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    red[2 * w] = r;
    red[2 * w + 1] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    r = 0.0;
    s = 0.0;
    for (int i = 0; i < nw; i++) {
      r += red[2 * i];
      s += red[2 * i + 1];
    }
  }
}

__device__ inline void st_f64(double *p, double v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long *>(p),
                     (unsigned long long)__double_as_longlong(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double ld_f64(const double *p) {
  return __longlong_as_double((long long)__hip_atomic_load(
      reinterpret_cast<const unsigned long long *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}

// Energy check at step count n: tile t adds its partial sums (r, s) (each
// thread's share); the last tile to arrive folds every tile's sums in tile
// order (deterministic for a given block size) and keeps the largest
// relative residual |sum r| / sum s of the checks.  Every thread of a tile
// block calls it.
__device__ inline void health_energy(const StepArgs &a, int t, double r, double s, long long n) {
  __shared__ double red[2 * 16];
  __shared__ int last;
  block_sum2(r, s, red);
  if (threadIdx.x == 0) {
    st_f64(a.hpart + 2 * t, r);
    st_f64(a.hpart + 2 * t + 1, s);
    __threadfence();
    last = __hip_atomic_fetch_add(&a.hl->done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
           (unsigned)(a.nt - 1);
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  r = 0.0;
  s = 0.0;
  for (int i = threadIdx.x; i < a.nt; i += blockDim.x) {
    r += ld_f64(a.hpart + 2 * i);
    s += ld_f64(a.hpart + 2 * i + 1);
  }
  block_sum2(r, s, red);
  if (threadIdx.x == 0) {
    Health *h = a.hl;
    const double rho = s > 0.0 ? fabs(r) / s : fabs(r);
    const double mx = ld_f64(&h->energy_max);
    if (!isnan(mx) && !(rho <= mx)) {
      st_f64(&h->energy_max, rho);
      __hip_atomic_store(&h->energy_step, n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __hip_atomic_fetch_add(&h->checks, 1LL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&h->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// per-node coefficients of the update
template <typename R>
struct NodeData {
  R alpha, beta, bA, bAT, beA, bTa, bP;
  int rec;
};

// coefficients of updated node j: alpha, beta from the LDS stage, the boundary
// record (if any) from global memory
template <typename R, bool TDC>
__device__ inline void load_node(const StepArgs &a, const R *La, const R *Lb, const int *Lr, int j,
                                 NodeData<R> &d) {
  d.alpha = La[j];
  d.beta = TDC ? Lb[j] : (R)0;
  const int r = Lr[j];
  d.rec = r;
  if (r >= 0) {
    d.bA = ((const R *)a.rA)[r];
    d.bAT = ((const R *)a.rAT)[r];
    d.beA = ((const R *)a.reA)[r];
    d.bTa = ((const R *)a.rTa)[r];
    d.bP = ((const R *)a.rP)[r];
  }
}

// Sum of the node's slots in ascending element order (Eq. 10-11), surface loads
// (Eq. 4, 5, 7) and the explicit update (Eq. 16): dT = (Q - F) / (alpha + beta T).
// Returns the new hi (and lo for the compensated mode).
template <typename R, int MODE, bool TDC>
__device__ inline R node_update(const NodeData<R> &d, int j, int maxinc, int stride, R T, float lo,
                                const R *slot, R Tz, const R *ctab, int nct, float &lo_new) {
#pragma clang fp contract(off)
  // the slots are read eight at a time (independent LDS reads in flight), then
  // added in position order; positions past the node's incidence hold zeros
  R F = 0;
  for (int p0 = 0; p0 < maxinc; p0 += 8) {
    R v[8];
#pragma unroll
    for (int p = 0; p < 8; p++) v[p] = p0 + p < maxinc ? slot[(p0 + p) * stride + j] : (R)0;
    if (p0 == 0) {
      F = v[0];
    } else {
      F += v[0];
    }
#pragma unroll
    for (int p = 1; p < 8; p++) F += v[p];
  }
  R Q = 0;
  if (d.rec >= 0) {
    R x = T - Tz, y = d.bTa - Tz;
    // (T-Tz)^4 - (Ta-Tz)^4 in factored form
    Q = (d.bAT - d.bA * T) - d.beA * ((T - d.bTa) * (x + y) * (x * x + y * y)) + d.bP;
  }
  R den = d.alpha;
  if (TDC) den = cap_den(d.alpha, d.beta, T, ctab, nct);
  const R dT = (Q - F) / den;
  if (MODE == 1) {
    // compensated accumulation: T = hi + lo, Fast2Sum of hi and (dT + lo)
    const float yv = (float)dT + lo;
    const float tv = (float)T + yv;
    lo_new = yv - (tv - (float)T);
    return (R)tv;
  }
  lo_new = 0.0f;
  return T + dT;
}

constexpr int kMaxBlock = 512;

// Element loads of elements [i0, i1) of the tile, EPT per thread at a time:
// all entry and operator loads are issued before the first element is
// evaluated.
template <typename R, int NE, bool TDK, bool GEN, int EPT>
__device__ inline void elements_from_global(const StepArgs &a, const TileHdr &th, int i0, int i1,
                                            const R *Tl, R *slot, int stride, int nupd,
                                            uint32_t pmask, const KLaw<R> &kl) {
  using EntT = typename Ent<NE>::T;
  const EntT *ent = reinterpret_cast<const EntT *>(a.ent);
  const R *Hb = (const R *)a.H;
  const int bs = blockDim.x;
  for (int base = i0 + threadIdx.x; base < i1; base += EPT * bs) {
    EntT w[EPT];
    R h[EPT][6];
#pragma unroll
    for (int q = 0; q < EPT; q++) {
      const int i = base + q * bs;
      if (i < i1) {
        const int64_t e = (int64_t)th.estart + i;
        w[q] = ent[e];
#pragma unroll
        for (int r = 0; r < 6; r++) h[q][r] = Hb[(int64_t)r * a.Eexp + e];
      }
    }
#pragma unroll
    for (int q = 0; q < EPT; q++)
      if (base + q * bs < i1)
        element_to_slots<R, NE, TDK>(w[q], h[q], Tl, slot, stride, nupd, a.pb, pmask,
                                     elem_law<GEN>(a, kl, (int64_t)th.estart + base + q * bs));
  }
}

// One launch advances the tile's owned nodes a.k steps (temporal blocking).
// MODE: 0 plain (R = float or double), 1 compensated FP32 (hi, lo pair).
// Memory round trips are batched: the first EPT elements of every thread are
// loaded before the T staging, the staging issues all its halo ids and then
// all values at once, and per-node coefficients come from LDS.  EPT, SPT and
// NPT are sized so that every variant fits 128 VGPRs (4 waves per SIMD)
// without spilling.
template <typename R, int NE, int MODE, bool TDK, bool TDC, bool GEN>
__global__ __launch_bounds__(kMaxBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_step(
    StepArgs a) {
  constexpr int EPT = NE == 8 ? (sizeof(R) == 4 ? 4 : 2) : (sizeof(R) == 4 ? 6 : 2);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int b = blockIdx.x;
  const int t = (b & 7) * a.nper + (b >> 3);
  if (t >= a.nt) return;  // whole block leaves before any barrier
  const TileHdr th = a.tiles[t];
  // level counts are read through global memory: a run-time index into the
  // local copy of the header would put the whole header in scratch
  const int32_t *cum_n = a.tiles[t].cum_n, *cum_e = a.tiles[t].cum_e;
  const int tid = threadIdx.x, bs = blockDim.x;
  const int k = a.k;
  const int nown = th.nown;
  const int nT = cum_n[k], nU = cum_n[k - 1], nE = cum_e[k - 1];
  using EntT = typename Ent<NE>::T;
  const EntT *ent = reinterpret_cast<const EntT *>(a.ent);
  const R *Hb = (const R *)a.H;
  // ---- first sub-step's elements: loads issued before the staging ----
  EntT ew[EPT];
  R eh[EPT][6];
#pragma unroll
  for (int q = 0; q < EPT; q++) {
    const int i = tid + q * bs;
    if (i < nE) {
      const int64_t e = (int64_t)th.estart + i;
      ew[q] = ent[e];
#pragma unroll
      for (int r = 0; r < 6; r++) eh[q][r] = Hb[(int64_t)r * a.Eexp + e];
    }
  }
  // ---- LDS: T of touched nodes; alpha, beta, record id, lo and slots of the
  // nodes the launch updates ----
  R *Tl = reinterpret_cast<R *>(smem_raw);
  R *La = Tl + nT;
  R *Lb = La + nU;
  int *Lr = reinterpret_cast<int *>(Lb + nU);
  float *Llo = reinterpret_cast<float *>(Lr + nU);
  R *slot = reinterpret_cast<R *>(Llo + (MODE == 1 ? nU : 0));
  if (sizeof(R) == 8)
    slot = reinterpret_cast<R *>((reinterpret_cast<uintptr_t>(slot) + 7) & ~uintptr_t(7));
  // table laws: the table's value at every touched node after the slots
  KLaw<R> kl = step_law<R, GEN>(a);
  const bool tabs = GEN && a.nkt > 0;
  if (tabs) kl.nv = slot + a.maxinc * nU;
  const R *Tin = (const R *)a.Tin;
  const R *alpha = (const R *)a.alpha, *beta = (const R *)a.beta;
  // SPT nodes per thread at a time: all halo ids, then all values
  constexpr int SPT = 4;
  for (int base = 0; base < nT; base += SPT * bs) {
    int gi[SPT];
#pragma unroll
    for (int q = 0; q < SPT; q++) {
      const int j = base + tid + q * bs;
      gi[q] = j < nown ? th.nstart + j : (j < nT ? a.halo[th.hstart + j - nown] : 0);
    }
    R tv[SPT], av[SPT], bv[SPT];
    float lv[SPT];
    int rv[SPT];
#pragma unroll
    for (int q = 0; q < SPT; q++) {
      const int j = base + tid + q * bs;
      if (j < nT) tv[q] = Tin[gi[q]];
      if (j < nU) {
        av[q] = alpha[gi[q]];
        if (TDC) bv[q] = beta[gi[q]];
        if (MODE == 1) lv[q] = a.loin[gi[q]];
        rv[q] = j < nown ? (j < th.nbnd ? th.bstart + j : -1) : a.rec_of[gi[q]];
      }
    }
#pragma unroll
    for (int q = 0; q < SPT; q++) {
      const int j = base + tid + q * bs;
      if (j < nT) {
        Tl[j] = tv[q];
        if (tabs) kl.stage(j, tv[q]);
      }
      if (j < nU) {
        La[j] = av[q];
        if (TDC) Lb[j] = bv[q];
        if (MODE == 1) Llo[j] = lv[q];
        Lr[j] = rv[q];
      }
    }
  }
  const int nslot = a.maxinc * nU;
  for (int j = tid; j < nslot; j += bs) slot[j] = (R)0;
  __syncthreads();
  const R Tz = (R)a.Tz;
  const uint32_t pmask = (1u << a.pb) - 1u;
  R *Tout = (R *)a.Tout;
  // Sub-step s updates the nodes of level <= k - s from the elements whose
  // lowest node level is <= k - s.  The first element phase (from the
  // prefetched registers) is peeled off so those registers die before the loop.
  {
    const int nU1 = cum_n[k - 1], nE1 = cum_e[k - 1];
#pragma unroll
    for (int q = 0; q < EPT; q++)
      if (tid + q * bs < nE1)
        element_to_slots<R, NE, TDK>(ew[q], eh[q], Tl, slot, nU, nU1, a.pb, pmask,
                                     elem_law<GEN>(a, kl, (int64_t)th.estart + tid + q * bs));
    elements_from_global<R, NE, TDK, GEN, EPT>(a, th, EPT * bs, nE1, Tl, slot, nU, nU1, pmask, kl);
  }
  __syncthreads();
  // health: the first sub-step at which an owned node of the wave left the
  // window (wave-uniform, a scalar register)
  int bad = 0;
  const R wlo = win_lo<R>(a), whi = win_hi<R>(a);
  for (int s = 1;; s++) {
    const int nUs = cum_n[k - s];
    const bool last = s == k;  // then nUs == nown
    bool out = false;
    // NPT nodes per thread at a time: coefficient and record loads first
    constexpr int NPT = sizeof(R) == 4 ? 4 : 1;
    for (int base = 0; base < nUs; base += NPT * bs) {
      NodeData<R> d[NPT];
#pragma unroll
      for (int q = 0; q < NPT; q++) {
        const int j = base + tid + q * bs;
        if (j < nUs) load_node<R, TDC>(a, La, Lb, Lr, j, d[q]);
      }
#pragma unroll
      for (int q = 0; q < NPT; q++) {
        const int j = base + tid + q * bs;
        if (j >= nUs) continue;
        const R T = Tl[j];
        const float lo = MODE == 1 ? Llo[j] : 0.0f;
        float lo_new;
        const R Tn = node_update<R, MODE, TDC>(d[q], j, a.maxinc, nU, T, lo, slot, Tz,
                                               GEN ? (const R *)a.ctab : nullptr, GEN ? a.nct : 0,
                                               lo_new);
        // owned nodes (the others are checked by their owners)
        out = out || (j < nown && outside(Tn, wlo, whi));
        if (last) {
          Tout[th.nstart + j] = Tn;
          if (MODE == 1) a.loout[th.nstart + j] = lo_new;
        } else {
          Tl[j] = Tn;
          if (tabs) kl.stage(j, Tn);
          if (MODE == 1) Llo[j] = lo_new;
        }
      }
    }
    if (!bad && __ballot(out)) bad = s;
    if (last) {
      if (a.hl && bad && (tid & 63) == 0) health_bad(a, health_step0(a) + bad);
      break;
    }
    __syncthreads();
    const int nUn = cum_n[k - s - 1], nEn = cum_e[k - s - 1];
    elements_from_global<R, NE, TDK, GEN, EPT>(a, th, 0, nEn, Tl, slot, nU, nUn, pmask, kl);
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// One-step kernel: launches that advance a single step.  Same arithmetic as
// k_step with k = 1, arranged for the shortest chain of memory round trips on
// a lightly occupied chip: the entries and operators of the first EPT elements
// and the coefficients of the first NPT nodes of every thread are loaded
// before the T staging, there is no sub-step loop to keep them alive across,
// and the compiler keeps the FP32 variants within 128 VGPRs.
#ifndef FED_FASTDIV
#define FED_FASTDIV 1
#endif

template <typename R>
struct Node1 {
  R alpha, beta, bA, bAT, beA, bTa, bP;
  float lo;
};

template <typename R, int MODE, bool TDC>
__device__ inline void load_node1(const StepArgs &a, const TileHdr &th, int j, Node1<R> &d) {
  const int k = th.nstart + j;
  d.alpha = ((const R *)a.alpha)[k];
  d.beta = TDC ? ((const R *)a.beta)[k] : (R)0;
  d.lo = MODE == 1 ? a.loin[k] : 0.0f;
  if (j < th.nbnd) {
    const int r = th.bstart + j;
    d.bA = ((const R *)a.rA)[r];
    d.bAT = ((const R *)a.rAT)[r];
    d.beA = ((const R *)a.reA)[r];
    d.bTa = ((const R *)a.rTa)[r];
    d.bP = ((const R *)a.rP)[r];
  }
}

// (Q - F) / den; in FP32 with the hardware reciprocal-based quotient (a few
// ulp, far below the compensated state's resolution of the increment)
template <typename R>
__device__ inline R quotient(R num, R den) {
  return num / den;
}
template <>
__device__ inline float quotient<float>(float num, float den) {
#if FED_FASTDIV
  return __fdividef(num, den);
#else
  return num / den;
#endif
}

// Surface loads (Eq. 4, 5, 7) and the explicit update (Eq. 16) of one node with
// temperature T (hi) and conductive load F: dT = (Q - F) / (alpha + beta T).
// Returns the new hi; lo_new receives the new lo of the compensated mode.
template <typename R, int MODE, bool TDC>
__device__ inline R advance(const Node1<R> &d, bool bnd, R T, R F, R Tz, const R *ctab, int nct,
                           float &lo_new, R &Qo, R &deno) {
#pragma clang fp contract(off)
  R Q = 0;
  if (bnd) {
    R x = T - Tz, y = d.bTa - Tz;
    // (T-Tz)^4 - (Ta-Tz)^4 in factored form
    Q = (d.bAT - d.bA * T) - d.beA * ((T - d.bTa) * (x + y) * (x * x + y * y)) + d.bP;
  }
  R den = d.alpha;
  if (TDC) den = cap_den(d.alpha, d.beta, T, ctab, nct);
  Qo = Q;
  deno = den;
  const R dT = quotient<R>(Q - F, den);
  if (MODE == 1) {
    // compensated accumulation: T = hi + lo, Fast2Sum of hi and (dT + lo)
    const float yv = (float)dT + d.lo;
    const float tv = (float)T + yv;
    lo_new = yv - (tv - (float)T);
    return (R)tv;
  }
  lo_new = 0.0f;
  return T + dT;
}

// conductive load of owned node j: its slots summed in position (= ascending
// element) order
template <typename R>
__device__ inline R slot_sum(const R *slot, int j, int nown, int maxinc) {
  R F = slot[j];
  for (int p = 1; p < maxinc; p++) F += slot[p * nown + j];
  return F;
}

// bad: the new temperature is outside the health window; r, s: the node's
// energy terms (when the launch checks the energy balance)
template <typename R, int MODE, bool TDC, bool GEN>
__device__ inline void update1(const StepArgs &a, const TileHdr &th, int j, const Node1<R> &d,
                               const R *Tl, const R *slot, R Tz, bool &bad, double &r, double &s) {
  const int k = th.nstart + j;
  const R F = slot_sum(slot, j, th.nown, a.maxinc);
  float lo_new;
  R Q, den;
  const R T0 = Tl[j];
  const R hi = advance<R, MODE, TDC>(d, j < th.nbnd, T0, F, Tz, GEN ? (const R *)a.ctab : nullptr,
                                     GEN ? a.nct : 0, lo_new, Q, den);
  ((R *)a.Tout)[k] = hi;
  if (MODE == 1) a.loout[k] = lo_new;
  if (outside(hi, win_lo<R>(a), win_hi<R>(a))) bad = true;
  if (a.energy) energy_terms<R, MODE>(den, Q, F, T0, d.lo, hi, lo_new, r, s);
}

template <typename R, int NE, int MODE, bool TDK, bool TDC, bool GEN, int OP = 0>
__global__ __launch_bounds__(1024) void k_step1(StepArgs a) {
  constexpr int HW = Op<R, NE, OP>::W;  // operator values per element
  constexpr int EPT = OP >= 1 ? 1
                      : NE == 8 ? (sizeof(R) == 4 ? 4 : 2) : (sizeof(R) == 4 ? (TDK ? 6 : 8) : 3);
  constexpr int NPT = OP >= 1 ? (sizeof(R) == 4 ? 2 : 1) : (sizeof(R) == 4 ? 4 : 2);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int b = blockIdx.x;
  const int t = (b & 7) * a.nper + (b >> 3);
  if (t >= a.nt) return;  // whole block leaves before any barrier
  const TileHdr th = a.tiles[t];
  const int nE = a.tiles[t].cum_e[0];            // elements touching owned nodes
  const int nhalo = a.tiles[t].cum_n[1] - th.nown;  // first halo ring
  const int tid = threadIdx.x, bs = blockDim.x;
  const int nown = th.nown, ntouch = nown + nhalo;
  using EntT = typename Ent<NE>::T;
  const EntT *ent = reinterpret_cast<const EntT *>(a.ent);
  const R *Hb = (const R *)a.H;
  // ---- T-independent loads ----
  EntT ew[EPT];
  R eh[EPT][HW];
#pragma unroll
  for (int q = 0; q < EPT; q++) {
    const int i = tid + q * bs;
    if (i < nE) {
      const int64_t e = (int64_t)th.estart + i;
      ew[q] = ld_entries(ent + e);
#pragma unroll
      for (int r = 0; r < HW; r++) eh[q][r] = ld_stream(Hb + (int64_t)r * a.Eexp + e);
    }
  }
  Node1<R> nd[NPT];
#pragma unroll
  for (int q = 0; q < NPT; q++) {
    const int j = tid + q * bs;
    if (j < nown) load_node1<R, MODE, TDC>(a, th, j, nd[q]);
  }
  // ---- stage T of owned and first-ring halo nodes; clear the slots ----
  // (table laws: the table's value at every touched node after the slots)
  R *Tl = reinterpret_cast<R *>(smem_raw);
  R *slot = Tl + ntouch;
  const int nslot = a.maxinc * nown;
  KLaw<R> kl = step_law<R, GEN>(a);
  const bool tabs = GEN && a.nkt > 0;
  if (tabs) kl.nv = slot + nslot;
  const R *Tin = (const R *)a.Tin;
  for (int j = tid; j < nown; j += bs) {
    const R v = Tin[th.nstart + j];
    Tl[j] = v;
    if (tabs) kl.stage(j, v);
  }
  for (int j = tid; j < nhalo; j += bs) {
    const R v = Tin[a.halo[th.hstart + j]];
    Tl[nown + j] = v;
    if (tabs) kl.stage(nown + j, v);
  }
  for (int j = tid; j < nslot; j += bs) slot[j] = (R)0;
  __syncthreads();
  // ---- element loads into the node-local slots ----
  const uint32_t pmask = (1u << a.pb) - 1u;
#pragma unroll
  for (int q = 0; q < EPT; q++)
    if (tid + q * bs < nE)
      element_to_slots<R, NE, TDK, OP>(ew[q], eh[q], Tl, slot, nown, nown, a.pb, pmask,
                                       elem_law<GEN>(a, kl, (int64_t)th.estart + tid + q * bs));
  for (int i = tid + EPT * bs; i < nE; i += bs) {
    const int64_t e = (int64_t)th.estart + i;
    R h[HW];
#pragma unroll
    for (int r = 0; r < HW; r++) h[r] = ld_stream(Hb + (int64_t)r * a.Eexp + e);
    element_to_slots<R, NE, TDK, OP>(ld_entries(ent + e), h, Tl, slot, nown, nown, a.pb, pmask,
                                     elem_law<GEN>(a, kl, e));
  }
  __syncthreads();
  // ---- per node: ordered sum, surface loads, explicit update ----
  const R Tz = (R)a.Tz;
  bool bad = false;
  double er = 0.0, es = 0.0;
#pragma unroll
  for (int q = 0; q < NPT; q++) {
    const int j = tid + q * bs;
    if (j < nown) update1<R, MODE, TDC, GEN>(a, th, j, nd[q], Tl, slot, Tz, bad, er, es);
  }
  for (int j = tid + NPT * bs; j < nown; j += bs) {
    Node1<R> d;
    load_node1<R, MODE, TDC>(a, th, j, d);
    update1<R, MODE, TDC, GEN>(a, th, j, d, Tl, slot, Tz, bad, er, es);
  }
  // ---- health: the window, and the energy balance at a check step ----
  if (a.hl) {
    const long long n = health_step0(a) + 1;
    if (bad) health_bad(a, n);
    if (a.energy) health_energy(a, t, er, es, n);
  }
}

template <typename R, int NE, int MODE, bool TDK, bool TDC, bool GEN, int OP = 0>
hipError_t step_t(const StepArgs &a, hipStream_t s) {
  if (a.k == 1)
    hipLaunchKernelGGL((k_step1<R, NE, MODE, TDK, TDC, GEN, OP>), dim3(8 * a.nper), dim3(a.block),
                       a.lds, s, a);
  else if (OP == 0)  // the host allows K > 1 with the folded operator only
    hipLaunchKernelGGL((k_step<R, NE, MODE, TDK, TDC, GEN>), dim3(8 * a.nper), dim3(a.block),
                       a.lds, s, a);
  return hipGetLastError();
}

template <typename R, int NE, int MODE, bool TDK, bool TDC, bool GEN, int OP = 0>
hipError_t step_attr(int bytes) {
  hipError_t e = hipFuncSetAttribute((const void *)k_step1<R, NE, MODE, TDK, TDC, GEN, OP>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess || OP != 0) return e;
  return hipFuncSetAttribute((const void *)k_step<R, NE, MODE, TDK, TDC, GEN>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

// tables or per-element laws run the general instance (T-dependent k and c,
// which covers every law); the others the instance of their linear law; the
// uniform-gradient hexahedron runs the general instance of its operator
template <typename R, int NE, int MODE>
hipError_t step_dispatch_tt(const StepArgs &a, hipStream_t s) {
  if (NE == 8 && a.op == 1) return step_t<R, 8, MODE, true, true, true, 1>(a, s);
  if (NE == 8 && a.op == 2) return step_t<R, 8, MODE, true, true, true, 2>(a, s);
  if (a.esk || a.ktab || a.ctab) return step_t<R, NE, MODE, true, true, true>(a, s);
  if (a.tdk)
    return a.tdc ? step_t<R, NE, MODE, true, true, false>(a, s) : step_t<R, NE, MODE, true, false, false>(a, s);
  return a.tdc ? step_t<R, NE, MODE, false, true, false>(a, s) : step_t<R, NE, MODE, false, false, false>(a, s);
}

template <typename R, int NE, int MODE>
hipError_t attr_dispatch_tt(int tdk, int tdc, int gen, int op, int bytes) {
  if (NE == 8 && op == 1) return step_attr<R, 8, MODE, true, true, true, 1>(bytes);
  if (NE == 8 && op == 2) return step_attr<R, 8, MODE, true, true, true, 2>(bytes);
  if (gen) return step_attr<R, NE, MODE, true, true, true>(bytes);
  if (tdk)
    return tdc ? step_attr<R, NE, MODE, true, true, false>(bytes) : step_attr<R, NE, MODE, true, false, false>(bytes);
  return tdc ? step_attr<R, NE, MODE, false, true, false>(bytes) : step_attr<R, NE, MODE, false, false, false>(bytes);
}

// ---------------------------------------------------------------------------
// Adjoint step (not in the paper: the exact transpose of the explicit step).
// The forward step of a node that is not Dirichlet is
//   T' = T + (Q(T) - F(T)) / den,  den = alpha + beta T  (= C / dt),
// F_e = s_e K0_e T_e with s_e = s0 + s1 Tbar_e, and Q holding convection
// -hA (T - Ta), radiation -sigma eps A ((T - Tz)^4 - (Ta - Tz)^4) and fixed
// inputs.  With mu = lambda^{n+1} / den (0 on Dirichlet nodes, den = +inf)
// and dT = T^{n+1} - T^n its transpose is
//   lambda^n_j = lambda_j - sum_{e owns j} [s_e (K0_e mu_e)_j + s1 / n_e (mu_e . K0_e T_e)]
//              - mu_j (hA_j + 4 sigma eps A_j (T_j - Tz)^3) - mu_j beta_j dT_j,
// (K0_e symmetric) and the parameter derivatives accumulated over the steps are
//   d/d log k_e : -s_e mu_e . K0_e T^n_e
//   d/d c_e     : -(rho V_e / n_e) sum_a mu_a dT_a / dt_a
//   d/d h_f     : -|f|/n_f sum_{k in f} mu_k (T^n_k - Ta_f)  (via S0, S1)
// The tile structure, the slot order of the nodal sums and the compensated
// pair are those of the forward step.
template <typename R, int NE>
struct ElemAdj;

template <typename R>
struct ElemAdj<R, 8> {
  __device__ static void u(const R *V, const uint32_t *loc, R &ux, R &uy, R &uz) {
    R T0 = V[loc[0]], T1 = V[loc[1]], T2 = V[loc[2]], T3 = V[loc[3]];
    R T4 = V[loc[4]], T5 = V[loc[5]], T6 = V[loc[6]], T7 = V[loc[7]];
    ux = ((T1 - T0) + (T2 - T3)) + ((T5 - T4) + (T6 - T7));
    uy = ((T3 - T0) + (T2 - T1)) + ((T7 - T4) + (T6 - T5));
    uz = ((T4 - T0) + (T5 - T1)) + ((T6 - T2) + (T7 - T3));
  }
};

template <typename R>
struct ElemAdj<R, 4> {
  __device__ static void u(const R *V, const uint32_t *loc, R &ux, R &uy, R &uz) {
    R T0 = V[loc[0]];
    ux = V[loc[1]] - T0;
    uy = V[loc[2]] - T0;
    uz = V[loc[3]] - T0;
  }
};

// mu_e . K0_e T_e of the uniform-gradient hexahedron (K0_e at s = 1); the
// folded operator computes it inline from the gradient sums
template <typename R, int NE, int OP>
struct AdjDot;
template <typename R>
struct AdjDot<R, 8, 1> {
  __device__ static R dot(const R *Lmu, const R *LT, const uint32_t *loc, const R *h) {
#pragma clang fp contract(off)
    // (Bbar mu)^T (V D) (Bbar T)
    R g[2][3] = {};
    const R *V2[2] = {Lmu, LT};
#pragma unroll
    for (int w = 0; w < 2; w++) {
      const R t7 = V2[w][loc[7]];
#pragma unroll
      for (int n = 0; n < 7; n++) {
        const R d = V2[w][loc[n]] - t7;
        g[w][0] += h[3 * n] * d;
        g[w][1] += h[3 * n + 1] * d;
        g[w][2] += h[3 * n + 2] * d;
      }
    }
    const R *vd = h + 21;
    const R qx = vd[0] * g[1][0] + vd[3] * g[1][1] + vd[5] * g[1][2];
    const R qy = vd[3] * g[1][0] + vd[1] * g[1][1] + vd[4] * g[1][2];
    const R qz = vd[5] * g[1][0] + vd[4] * g[1][1] + vd[2] * g[1][2];
    return g[0][0] * qx + g[0][1] * qy + g[0][2] * qz;
  }
};

// with hourglass control: the mean-gradient part plus kappa sum_alpha
// c_alpha(mu) c_alpha(T)
template <typename R>
struct AdjDot<R, 8, 2> {
  __device__ static R dot(const R *Lmu, const R *LT, const uint32_t *loc, const R *h) {
#pragma clang fp contract(off)
    R g[2][3] = {}, c[2][4];
    const R *V2[2] = {Lmu, LT};
#pragma unroll
    for (int w = 0; w < 2; w++) {
      const R t7 = V2[w][loc[7]];
      R d[7];
#pragma unroll
      for (int n = 0; n < 7; n++) {
        d[n] = V2[w][loc[n]] - t7;
        g[w][0] += h[3 * n] * d[n];
        g[w][1] += h[3 * n + 1] * d[n];
        g[w][2] += h[3 * n + 2] * d[n];
      }
      ElemMeanHg<R>::amps(d, g[w][0], g[w][1], g[w][2], h, c[w]);
    }
    const R *vd = h + 21;
    const R qx = vd[0] * g[1][0] + vd[3] * g[1][1] + vd[5] * g[1][2];
    const R qy = vd[3] * g[1][0] + vd[1] * g[1][1] + vd[4] * g[1][2];
    const R qz = vd[5] * g[1][0] + vd[4] * g[1][1] + vd[2] * g[1][2];
    R hg = 0;
#pragma unroll
    for (int al = 0; al < 4; al++) hg += c[0][al] * c[1][al];
    return (g[0][0] * qx + g[0][1] * qy + g[0][2] * qz) + h[27] * hg;
  }
};

// The arithmetic of the adjoint step, shared by the one-step and the resident
// kernels so that both round alike (no FMA contraction: the source fixes it).

// Per touched node at step n: mu = lambda^{n+1} / den(T^n) (0 on Dirichlet
// nodes, den = +inf), and w = mu (T^{n+1} - T^n) / dt dc/dc0 (dc/dc0 = 1, or the
// c table's value at T^n), the node's term of the capacity derivative.
template <typename R>
__device__ inline void adj_stage(R lam, R alpha, R beta, R tn, R tn1, R rdt, bool tdc,
                                 const R *ctab, int nct, R &mu, R &w) {
#pragma clang fp contract(off)
  const R den = tdc ? cap_den(alpha, beta, tn, ctab, nct) : alpha;
  mu = lam / den;
  R dcdc0 = (R)1, sl;
  if (nct) dcdc0 = table_eval(ctab, nct, tn, sl);
  w = mu * ((tn1 - tn) * rdt * dcdc0);
}

// Element part: F = s_e K0_e mu_e plus the conductivity-factor term
// d s_e / d T_a (mu_e . K0_e T_e) at every node a, s_e, mu_e . K0_e T_e (when
// needed) and the sum of w over the nodes.
template <typename R, int NE, int OP>
__device__ inline void adj_elem(const uint32_t *loc, const R *h, const KLaw<R> &kle, bool tdk,
                                bool owner, const R *Lmu, const R *LT, const R *Lw, R F[NE],
                                R &se, R &muKT, R &gsum) {
#pragma clang fp contract(off)
  // s_e from T^n, as in the forward load
  se = kle.s0;
  if (tdk) {
    R Te[NE];
#pragma unroll
    for (int n = 0; n < NE; n++) Te[n] = LT[loc[n]];
    se = kle.template elem<NE>(Te);
  }
  muKT = (R)0;
  if constexpr (OP == 0) {
    // the gradient sums of mu serve both mu . K0 T and the load K0 mu
    R mx, my, mz;
    ElemAdj<R, NE>::u(Lmu, loc, mx, my, mz);
    if (tdk || owner) {
      R tx, ty, tz;
      ElemAdj<R, NE>::u(LT, loc, tx, ty, tz);
      const R qx = fma(h[5], tz, fma(h[3], ty, h[0] * tx));
      const R qy = fma(h[4], tz, fma(h[1], ty, h[3] * tx));
      const R qz = fma(h[2], tz, fma(h[4], ty, h[5] * tx));
      muKT = fma(mz, qz, fma(my, qy, mx * qx));
    }
    // the forward element load applied to mu at factor s_e
    Elem<R, NE>::apply(se, h, mx, my, mz, F);
  } else {
    if (tdk || owner) muKT = AdjDot<R, NE, OP>::dot(Lmu, LT, loc, h);
    Op<R, NE, OP>::load(Lmu, loc, KLaw<R>{se, (R)0, nullptr, 0}, false, h, F);
  }
  // n_e d s_e / d T_a is the law's slope at node a: s1 for the linear law (the
  // same term at every node), the table's slope at T_a (taken here, not kept
  // from above, so the slopes hold no registers through the element work)
  const R spread = tdk && !kle.n ? kle.s1 * ((R)1 / (R)NE) * muKT : (R)0;
#pragma unroll
  for (int n = 0; n < NE; n++)
    F[n] = F[n] + (tdk && kle.n ? kle.slope(LT[loc[n]]) * ((R)1 / (R)NE) * muKT : spread);
  gsum = (R)0;
  if (owner) {
#pragma unroll
    for (int n = 0; n < NE; n++) gsum = gsum + Lw[loc[n]];
  }
}

// Per-step parameter derivatives of an owner element, accumulated in FP64.
template <typename R>
__device__ inline void adj_grad(double &gk, double &gc, R se, R muKT, R mV, R gsum) {
#pragma clang fp contract(off)
  gk = gk + -(double)se * (double)muKT;
  gc = gc + -(double)mV * (double)gsum;
}

// Node part: lambda^n - lambda^{n+1} of an owned node before the Dirichlet mask.
template <typename R>
__device__ inline R adj_node(R F, R mu, bool bnd, R rA, R reA, R tn, R tn1, R Tz, bool tdc,
                             R dden) {
#pragma clang fp contract(off)
  R d = -F;
  if (bnd) {
    const R x = tn - Tz;
    d = d - (rA + (R)4 * reA * (x * x * x)) * mu;
  }
  if (tdc) d = d - dden * (tn1 - tn) * mu;
  return d;
}

// Sums of mu and mu T^n of a boundary node (for the face derivatives).
template <typename R>
__device__ inline void adj_bnd(double &S0, double &S1, R mu, R tn) {
#pragma clang fp contract(off)
  S0 = S0 + (double)mu;
  S1 = S1 + (double)mu * (double)tn;
}

// lambda^n from lambda^{n+1} = (hi, lo) and d, zero on Dirichlet nodes.
template <typename R, int MODE>
__device__ inline R adj_lambda(R hi, float lo, R d, bool fixed, float &lo_new) {
#pragma clang fp contract(off)
  if (MODE == 1) {
    const float yv = (float)d + lo;
    const float tv = (float)hi + yv;
    lo_new = fixed ? 0.0f : yv - (tv - (float)hi);
    return fixed ? (R)0 : (R)tv;
  }
  lo_new = 0.0f;
  return fixed ? (R)0 : hi + d;
}

// d den / dT: beta, or alpha times the c table's slope at T^n
template <typename R>
__device__ inline R adj_dden(R alpha, R beta, R tn, const R *ctab, int nct) {
  if (!nct) return beta;
  R sl;
  (void)table_eval(ctab, nct, tn, sl);
  return alpha * sl;
}

// GEN: the instance for property tables and per-element laws; the others
// compile the shared linear laws only (no table code, fewer registers)
template <typename R, int NE, int MODE, int OP = 0, bool GEN = true>
__global__ __launch_bounds__(1024) void k_adjoint1(AdjArgs a) {
  constexpr int HW = Op<R, NE, OP>::W;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int b = blockIdx.x;
  const int t = (b & 7) * a.nper + (b >> 3);
  if (t >= a.nt) return;
  const TileHdr th = a.tiles[t];
  const int nE = a.tiles[t].cum_e[0];
  const int nhalo = a.tiles[t].cum_n[1] - th.nown;
  const int tid = threadIdx.x, bs = blockDim.x;
  const int nown = th.nown, ntouch = nown + nhalo;
  // LDS: mu, T^n and w of touched nodes, slots of owned nodes
  R *Lmu = reinterpret_cast<R *>(smem_raw);
  R *LT = Lmu + ntouch;
  R *Lw = LT + ntouch;
  R *slot = Lw + ntouch;
  const R *lam = (const R *)a.lamin, *alpha = (const R *)a.alpha, *rdt = (const R *)a.rdt;
  const R *beta = (const R *)a.beta;
  const R *Tn = (const R *)a.Tn, *Tn1 = (const R *)a.Tn1;
  const bool tdk = a.tdk != 0, tdc = a.tdc != 0;
  const R *ctab = GEN ? (const R *)a.ctab : nullptr;
  const int nct = GEN ? a.nct : 0;
  for (int j = tid; j < ntouch; j += bs) {
    const int g = j < nown ? th.nstart + j : a.halo[th.hstart + j - nown];
    const R tn = Tn[g];
    adj_stage<R>(lam[g], alpha[g], tdc ? beta[g] : (R)0, tn, Tn1[g], rdt[g], tdc, ctab, nct,
                 Lmu[j], Lw[j]);
    LT[j] = tn;
  }
  const int nslot = a.maxinc * nown;
  for (int j = tid; j < nslot; j += bs) slot[j] = (R)0;
  __syncthreads();
  using EntT = typename Ent<NE>::T;
  const EntT *ent = reinterpret_cast<const EntT *>(a.ent);
  const R *Hb = (const R *)a.H;
  const R *mV = (const R *)a.mV;
  const KLaw<R> kl = GEN ? KLaw<R>{(R)a.s0, (R)a.s1, (const R *)a.ktab, a.nkt}
                         : KLaw<R>{(R)a.s0, (R)a.s1, nullptr, 0};
  const uint32_t pmask = (1u << a.pb) - 1u;
  for (int i = tid; i < nE; i += bs) {
    const int64_t e = (int64_t)th.estart + i;
    R h[HW];
#pragma unroll
    for (int r = 0; r < HW; r++) h[r] = ld_stream(Hb + (int64_t)r * a.Eexp + e);
    const EntT w = ld_entries(ent + e);
    uint32_t v[NE], loc[NE];
    Ent<NE>::unpack(w, v);
#pragma unroll
    for (int n = 0; n < NE; n++) loc[n] = v[n] >> a.pb;
    const bool owner = a.eowner[e] != 0;
    R F[NE], se, muKT, gsum;
    adj_elem<R, NE, OP>(loc, h, elem_law<GEN>(a, kl, e), tdk, owner, Lmu, LT, Lw, F, se, muKT,
                        gsum);
#pragma unroll
    for (int n = 0; n < NE; n++)
      if (loc[n] < (uint32_t)nown) slot[(v[n] & pmask) * nown + loc[n]] = F[n];
    if (owner) {
      const int32_t eo = a.eorig[e];
      double gk = a.g_logk[eo], gc = a.g_c[eo];
      adj_grad<R>(gk, gc, se, muKT, mV[eo], gsum);
      a.g_logk[eo] = gk;
      a.g_c[eo] = gc;
    }
  }
  __syncthreads();
  const R *rA = (const R *)a.rA, *reA = (const R *)a.reA;
  const R Tz = (R)a.Tz;
  R *lout = (R *)a.lamout;
  for (int j = tid; j < nown; j += bs) {
    const int k = th.nstart + j;
    const R F = slot_sum(slot, j, nown, a.maxinc);
    const R mu = Lmu[j], tn = LT[j], tn1 = Tn1[k];
    const bool bnd = j < th.nbnd;
    const int r = th.bstart + j;
    const R dden = tdc ? adj_dden<R>(alpha[k], beta[k], tn, ctab, nct) : (R)0;
    const R d = adj_node<R>(F, mu, bnd, bnd ? rA[r] : (R)0, bnd ? reA[r] : (R)0, tn, tn1, Tz, tdc,
                            dden);
    if (bnd) {
      double S0 = a.S0[r], S1 = a.S1[r];
      adj_bnd<R>(S0, S1, mu, tn);
      a.S0[r] = S0;
      a.S1[r] = S1;
    }
    float lo_new;
    lout[k] = adj_lambda<R, MODE>(lam[k], MODE == 1 ? a.lamloin[k] : 0.0f, d,
                                  alpha[k] == (R)INFINITY, lo_new);
    if (MODE == 1) a.lamloout[k] = lo_new;
  }
}

__global__ void k_face_grad(int64_t nf, int nfn, const int32_t *faces, const int32_t *perm,
                            const int32_t *rec_of, const double *farea, const double *fTa,
                            const double *S0, const double *S1, double *g_h) {
  int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (f >= nf) return;
  double ta = fTa ? fTa[f] : 0.0, acc = 0;
  for (int b = 0; b < nfn; b++) {
    int r = rec_of[perm[faces[f * nfn + b]]];
    acc += S1[r] - ta * S0[r];
  }
  g_h[f] = -farea[f] / nfn * acc;
}

template <typename R>
__global__ void k_adjoint_coefs(int64_t N, int64_t E, int ne, const double *dt_inst,
                                const int32_t *node_inst, const MatDev *mats, const int32_t *emat,
                                const double *V, R *rdt, R *mV) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < N) rdt[i] = (R)(1.0 / dt_inst[node_inst ? node_inst[i] : 0]);
  if (i < E) mV[i] = (R)(mats[emat ? emat[i] : 0].rho * V[i] / ne);
}

// caller order <-> internal order, FP64 in the caller's arrays
template <typename R, int MODE>
__global__ void k_set_T(int64_t N, const double *Tuser, const int32_t *perm, R *T, float *lo) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= N) return;
  double v = Tuser[k];
  int32_t ki = perm[k];
  R hv = (R)v;
  T[ki] = hv;
  if (MODE == 1) lo[ki] = (float)(v - (double)hv);
}

template <typename R, int MODE>
__global__ void k_set_dir(int64_t ndir, const int32_t *node, const double *val, R *T, float *lo) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= ndir) return;
  double v = val[i];
  R hv = (R)v;
  T[node[i]] = hv;
  if (MODE == 1) lo[node[i]] = (float)(v - (double)hv);
}

template <typename R, int MODE>
__global__ void k_get_T(int64_t N, const int32_t *perm, const R *T, const float *lo, double *Tuser) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= N) return;
  int32_t ki = perm[k];
  double v = (double)T[ki];
  if (MODE == 1) v += (double)lo[ki];
  Tuser[k] = v;
}

template <typename R, int MODE>
__global__ void k_check(int64_t N, const R *T, const float *lo, double lo_b, double hi_b, int *flag) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= N) return;
  double v = (double)T[k];
  if (MODE == 1) v += (double)lo[k];
  if (!(v >= lo_b && v <= hi_b)) atomicOr(flag, 1);  // also catches NaN
}

// health record: op 0 resets it, op 1 sets the graph replays' base step count
// to v, op 2 advances it by v (the last node of a captured graph), op 3
// clears the out-of-window record (a new window)
__global__ void k_health(Health *h, int op, long long v) {
  if (op == 3) {
    h->first_bad = ~0ull;
  } else if (op == 0) {
    h->first_bad = ~0ull;
    h->base = 0;
    h->energy_max = 0.0;
    h->energy_step = -1;
    h->checks = 0;
    h->done = 0;
  } else if (op == 1) {
    h->base = v;
  } else {
    h->base += v;
  }
}

// Order-preserving unsigned key of a double (larger key, larger value).
__device__ inline unsigned long long order_key(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

// Smallest and largest temperature (hi + lo) as order keys in keys[0], keys[1]
// (block reduction, then one atomic per block); *nan set if any is not finite.
template <typename R, int MODE>
__global__ void k_range(int64_t N, const R *T, const float *lo, unsigned long long *keys, int *nan) {
  __shared__ unsigned long long smin[1024 / 64], smax[1024 / 64];
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  unsigned long long kmin = ~0ull, kmax = 0ull;
  if (k < N) {
    double v = (double)T[k];
    if (MODE == 1) v += (double)lo[k];
    if (!isfinite(v)) atomicOr(nan, 1);
    kmin = kmax = order_key(v);
  }
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned long long a = __shfl_down(kmin, off, 64), b = __shfl_down(kmax, off, 64);
    kmin = a < kmin ? a : kmin;
    kmax = b > kmax ? b : kmax;
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    smin[w] = kmin;
    smax[w] = kmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < (int)(blockDim.x >> 6); i++) {
      kmin = smin[i] < kmin ? smin[i] : kmin;
      kmax = smax[i] > kmax ? smax[i] : kmax;
    }
    atomicMin(&keys[0], kmin);
    atomicMax(&keys[1], kmax);
  }
}

__global__ void k_permute(int eb, int64_t N, const int32_t *perm, const unsigned char *src,
                          unsigned char *dst, int to_internal) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= N) return;
  int64_t ki = perm[k];
  const unsigned char *s = src + (to_internal ? k : ki) * eb;
  unsigned char *d = dst + (to_internal ? ki : k) * eb;
  for (int i = 0; i < eb; i++) d[i] = s[i];
}

// ---------------------------------------------------------------------------
// Resident stepping.  One launch advances r.nsteps steps, with
// every tile's workgroup resident for the whole launch.  A tile keeps its
// elements' entries and operators and its nodes' coefficients and state in
// registers, so a step reads from memory only the halo temperatures and
// writes only the exported ones (owned nodes in another tile's halo).
// Step s >= 1 reads the halo from exchange buffer X[s & 1], polling each word
// until it carries tag0 + s; step s writes its exports, tagged tag0 + s + 1, to
// X[(s + 1) & 1]; step 0 reads the halo from the state Tin.  A word a reader
// finds with the tag it wants was written after the writer's tile had read
// every value it needed from the reader's tile for the previous step (each
// tile reads at least one value of every neighbour, and the relation is
// symmetric: an element joins an owned node of each tile), so a buffer is
// never overwritten while still in use and no flags or fences are needed.
// Tags grow from launch to launch, so a stale word never matches.  The element
// loads, the ordered nodal sums and the update are those of k_step1 on the
// same tiles, so both give bitwise-identical temperatures.

// Resident stepping compares the running extremes of every step's
// temperatures with the health window every kResCheck steps (a ballot a step
// measured ~0.14 us on a ~2.3 us step); the first step outside is then
// reported at the check that finds it, at most kResCheck - 1 steps late.
constexpr int kResCheck = 32;

// register capacity per thread: elements, owned nodes, halo ids
template <typename R, int NE>
struct ResCap {
  static constexpr int EPT = NE == 8 ? 2 : (sizeof(R) == 4 ? 8 : 4);
  static constexpr int NPT = NE == 8 ? 2 : 1;
  static constexpr int HPT = 2;
};

// Makes the packed entries opaque to the optimiser once per step, so it keeps
// them packed in registers instead of hoisting their unpacked form (four times
// the registers) out of the step loop.  Emits no instruction.
__device__ inline void keep_packed(uint4 &w) {
  uint32_t x = w.x, y = w.y, z = w.z, v = w.w;
  asm volatile("" : "+v"(x), "+v"(y), "+v"(z), "+v"(v));
  w = make_uint4(x, y, z, v);
}
__device__ inline void keep_packed(uint2 &w) {
  uint32_t x = w.x, y = w.y;
  asm volatile("" : "+v"(x), "+v"(y));
  w = make_uint2(x, y);
}

// LDS addresses as 32-bit integers (the local address space), so a kernel can
// keep precomputed addresses in registers and access LDS with no arithmetic
template <typename R>
using LdsPtr = __attribute__((address_space(3))) R *;
template <typename R>
__device__ inline uint32_t lds_addr(R *p) {
  return (uint32_t)(uintptr_t)(LdsPtr<R>)p;
}
template <typename R>
__device__ inline R lds_ld(uint32_t a) {
  return *(LdsPtr<R>)(uintptr_t)a;
}
template <typename R>
__device__ inline void lds_st(uint32_t a, R v) {
  *(LdsPtr<R>)(uintptr_t)a = v;
}

// 64-bit loads and stores, single-copy atomic and coherent across the XCDs'
// L2 caches
__device__ inline unsigned long long ld_word(const unsigned long long *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_word(unsigned long long *p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline unsigned long long tagged(unsigned tag, uint32_t bits) {
  return ((unsigned long long)tag << 32) | bits;
}

// tagged words of one value: one 64-bit (tag, value) word for float; one
// 16-byte word for double (below)
template <typename R>
struct Words;
// (ld: the raw words; ok: they carry `tag`; val: the value they hold)
template <>
struct Words<float> {
  static constexpr int W = 1;
  struct Raw {
    unsigned long long w;
  };
  __device__ static void put(unsigned long long *X, int k, unsigned tag, float v) {
    st_word(X + k, tagged(tag, __float_as_uint(v)));
  }
  __device__ static Raw ld(const unsigned long long *X, int k) { return Raw{ld_word(X + k)}; }
  __device__ static bool ok(const Raw &r, unsigned tag) { return (unsigned)(r.w >> 32) == tag; }
  __device__ static float val(const Raw &r) { return __uint_as_float((uint32_t)r.w); }
};
// FP64: one 16-byte word per value, (tag, low half, high half, tag), loaded
// and stored with one 128-bit access (half the memory requests of two 64-bit
// words).  Accesses are device-coherent (sc1); the load is volatile so every
// poll reads memory.  A reader accepts a word only when both tags match, so a
// store seen in part (its first or its last bytes only) is never taken.
template <>
struct Words<double> {
  static constexpr int W = 2;
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  struct Raw {
    u32x4 v;
  };
  __device__ static __amdgpu_buffer_rsrc_t rsrc(const unsigned long long *X) {
    // raw buffer over X (dword 3: the gfx9 buffer format); offsets stay below 2^31
    return __builtin_amdgcn_make_buffer_rsrc((void *)X, 0, 0x7fffffff, 0x00020000);
  }
  __device__ static void put(unsigned long long *X, int k, unsigned tag, double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const u32x4 d = {tag, (unsigned)b, (unsigned)(b >> 32), tag};
    __builtin_amdgcn_raw_buffer_store_b128(d, rsrc(X), k * 16, 0, /*sc1*/ 16);
  }
  __device__ static Raw ld(const unsigned long long *X, int k) {
    return Raw{__builtin_amdgcn_raw_buffer_load_b128(rsrc(X), k * 16, 0, /*sc1, volatile*/ 16 | (1u << 31))};
  }
  __device__ static bool ok(const Raw &r, unsigned tag) { return r.v[0] == tag && r.v[3] == tag; }
  __device__ static double val(const Raw &r) {
    return __longlong_as_double((long long)(((unsigned long long)r.v[2] << 32) | r.v[1]));
  }
};

// Polls a thread's halo words until each carries `want`, the values into hv.
// A poll issues the loads of all the thread's missing words before it looks
// at any, so it costs one memory round trip.  Gives up after spin_limit
// polls, or soon after another wave gave up, and sets *err.
template <typename R, int HPT>
__device__ inline void wait_halo(const unsigned long long *X, const int *hid, int nleft, int bs,
                                 unsigned want, R *hv, int spin_limit, int *err) {
  unsigned missing = 0;
#pragma unroll
  for (int q = 0; q < HPT; q++)
    if (q * bs < nleft) missing |= 1u << q;
  for (int it = 0; missing; it++) {
    typename Words<R>::Raw w[HPT];
#pragma unroll
    for (int q = 0; q < HPT; q++)
      if ((missing >> q) & 1u) w[q] = Words<R>::ld(X, hid[q]);
#pragma unroll
    for (int q = 0; q < HPT; q++)
      if (((missing >> q) & 1u) && Words<R>::ok(w[q], want)) {
        hv[q] = Words<R>::val(w[q]);
        missing &= ~(1u << q);
      }
    if (!missing) return;
    if (it >= spin_limit ||
        ((it & 255) == 255 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
      __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
    __builtin_amdgcn_s_sleep(1);
  }
}

// OP: the element operator (0 the folded 3x3, kept in registers for the whole
// launch; 1 and 2 the uniform-gradient hexahedron without and with hourglass
// control, 27 and 40 values an element, too many for registers: each step
// reads them again from memory, where the launch's repeated reads of the
// same data are served by the caches, and keeps only the packed entries)
template <typename R, int NE, int MODE, bool TDK, bool TDC, bool GEN, int OP = 0>
__global__ __launch_bounds__(1024) void k_resident(StepArgs a, ResArgs r) {
  constexpr int EPT = ResCap<R, NE>::EPT, NPT = ResCap<R, NE>::NPT, HPT = ResCap<R, NE>::HPT;
  constexpr int HW = Op<R, NE, OP>::W;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int b = blockIdx.x;
  const int t = (b & 7) * a.nper + (b >> 3);
  if (t >= a.nt) return;  // no tile: nobody reads from it
  const TileHdr th = a.tiles[t];
  const int nE = a.tiles[t].cum_e[0];
  const int nhalo = a.tiles[t].cum_n[1] - th.nown;
  const int tid = threadIdx.x, bs = blockDim.x;
  const int nown = th.nown, ntouch = nown + nhalo;
  using EntT = typename Ent<NE>::T;
  // (PRE with LDS positions: the entries that carry them)
  constexpr bool PRE0 = NE == 8 && sizeof(R) == 4 && OP == 0 && !GEN;
  const EntT *ent =
      reinterpret_cast<const EntT *>(PRE0 && r.sigma ? r.ent_sigma : a.ent);
  const R *Hb = (const R *)a.H;
  EntT ew[EPT];
  R eh[EPT][OP ? 1 : 6];
#pragma unroll
  for (int q = 0; q < EPT; q++) {
    const int i = tid + q * bs;
    if (i < nE) {
      const int64_t e = (int64_t)th.estart + i;
      ew[q] = ent[e];
      if constexpr (OP == 0) {
#pragma unroll
        for (int c = 0; c < 6; c++) eh[q][c] = Hb[(int64_t)c * a.Eexp + e];
      }
    }
  }
  // OPH: the FP32 uniform-gradient hexahedron without hourglass control, with
  // the shared laws, keeps the operators of the elements that touch the halo
  // in LDS (below); the other instances keep one code path, which their
  // registers need.
  // Hexahedra use node-major slots (below), except where the LDS is wanted
  // for more: the OPH operators, the FP64 uniform-gradient hexahedron (whose
  // tiles on distorted meshes touch more halo nodes than such slots leave LDS
  // for) and the FP64 general laws (their table values); they keep slots for
  // the owned nodes only.  FP32 hexahedra with the folded operator and the
  // shared linear laws keep precomputed LDS addresses instead of the packed
  // entries, the node temperatures' and the slots' (16 registers an element),
  // so the element phase spends no instructions on addressing (tables and
  // per-element laws need those registers)
  constexpr bool OPH = OP == 1 && !GEN && sizeof(R) == 4;
  constexpr bool NM =
      NE == 8 && (OP == 0 || (sizeof(R) == 4 && !OPH)) && !(GEN && sizeof(R) == 8);
  constexpr bool PRE = NM && sizeof(R) == 4 && OP == 0 && !GEN;
  const int nslot = NM ? ntouch * ((1 << a.pb) + 1) : a.maxinc * nown;
  R *Tl = reinterpret_cast<R *>(smem_raw);
  R *slot = Tl + ntouch;
  R *Lbnd = slot + nslot;  // [5][nbnd]: hA, hA Ta, sigma eps A, radiation Ta, power
  // table laws: the table's value at every touched node, staged with T
  const bool tabs = GEN && a.nkt > 0 && r.nvals;
  R *NV = Lbnd + 5 * th.nbnd;
  // the elements with every node owned come first in the tile's list
  const int nint = r.split ? th.nint : 0;
  // OPH: the operators of the elements that touch the halo, copied to LDS
  // once (element-major, an odd stride: the lanes of a wave read distinct
  // banks), so the elements that run after the halo wait read no memory; the
  // others read theirs from memory while the halo arrives
  constexpr int HWS = HW | 1;
  R *oph = NV + (tabs ? ntouch : 0);
  if constexpr (OPH) {
    if (r.ophalo) {
      const int nh = nE - nint;
      for (int k = tid; k < HW * nh; k += bs) {
        const int c = k / nh, m = k - c * nh;
        oph[m * HWS + c] = Hb[(int64_t)c * a.Eexp + th.estart + nint + m];
      }
    }
  }
  // PRE: a touched node's temperature and slots sit at LDS position sig(local
  // index) (r.sigma: the tile's touched nodes in caller order; the elements'
  // packed entries, r.ent_sigma, carry those positions already), the others
  // at the local index itself
  const int16_t *sg = PRE && r.sigma ? r.sigma + (int64_t)t * r.sstride : nullptr;
  auto sig = [&](int l) -> int { return PRE && sg ? (int)sg[l] : l; };
  uint32_t ta[PRE ? EPT : 1][8], sa[PRE ? EPT : 1][8];
  if constexpr (PRE) {
    const uint32_t tb = lds_addr(Tl), sb = lds_addr(slot);
#pragma unroll
    for (int q = 0; q < EPT; q++) {
      uint32_t v[8];
      Ent<8>::unpack(*reinterpret_cast<const uint4 *>(&ew[q]), v);
#pragma unroll
      for (int n = 0; n < 8; n++) {
        const uint32_t loc = v[n] >> a.pb;
        ta[q][n] = tb + loc * (uint32_t)sizeof(R);
        sa[q][n] = sb + (v[n] + loc) * (uint32_t)sizeof(R);
        // opaque from here on: the loop uses the whole addresses as they are
        // instead of re-adding the LDS bases at every access
        asm volatile("" : "+v"(ta[q][n]), "+v"(sa[q][n]));
      }
    }
  }
  const R *Tin = (const R *)a.Tin;
  // per owned node in registers: alpha, beta, lo, hi, exported; the boundary
  // records (5 coefficients of the first nbnd nodes) live in LDS
  R al[NPT], be[NPT], hi[NPT];
  float lo[NPT];
  bool ex[NPT];
#pragma unroll
  for (int q = 0; q < NPT; q++) {
    const int j = tid + q * bs;
    ex[q] = false;
    if (j < nown) {
      const int k = th.nstart + j;
      al[q] = ((const R *)a.alpha)[k];
      be[q] = TDC ? ((const R *)a.beta)[k] : (R)0;
      lo[q] = MODE == 1 ? a.loin[k] : 0.0f;
      hi[q] = Tin[k];
      ex[q] = r.exported[k] != 0;
    }
  }
  int hid[HPT];
#pragma unroll
  for (int q = 0; q < HPT; q++) {
    const int j = tid + q * bs;
    hid[q] = j < nhalo ? a.halo[th.hstart + j] : 0;
  }
  // PRE: LDS positions of this thread's owned and halo nodes, kept in
  // registers (the other instances use the local index itself)
  int jpos[PRE ? NPT : 1], hpos[PRE ? HPT : 1];
  if constexpr (PRE) {
#pragma unroll
    for (int q = 0; q < NPT; q++) jpos[q] = tid + q * bs < nown ? sig(tid + q * bs) : 0;
#pragma unroll
    for (int q = 0; q < HPT; q++) hpos[q] = tid + q * bs < nhalo ? sig(nown + tid + q * bs) : 0;
  }
  // the boundary records of the owned nodes into LDS (slots: NM above)
  const int nbnd = th.nbnd;
  for (int j = tid; j < nbnd; j += bs) {
    const int rr = th.bstart + j;
    Lbnd[j] = ((const R *)a.rA)[rr];
    Lbnd[nbnd + j] = ((const R *)a.rAT)[rr];
    Lbnd[2 * nbnd + j] = ((const R *)a.reA)[rr];
    Lbnd[3 * nbnd + j] = ((const R *)a.rTa)[rr];
    Lbnd[4 * nbnd + j] = ((const R *)a.rP)[rr];
  }
  // slots past a node's incidence are never written and stay zero
  for (int j = tid; j < nslot; j += bs) slot[j] = (R)0;
  KLaw<R> kl = step_law<R, GEN>(a);
  if (tabs) kl.nv = NV;
  const uint32_t dnv = (uint32_t)((NV - Tl) * (int)sizeof(R));  // byte offset T -> table value
  const R Tz = (R)a.Tz;
  const uint32_t pmask = (1u << a.pb) - 1u;
  int prow = r.pts_row;
  // element loads into the node-local slots
  // (materials with different k(T) laws: the element's own (s0, s1), read
  // when the element runs, as in the one-step kernel)
  // the operator of element slot q from memory (SoA, coalesced).  The offset
  // is made opaque on every call, so the compiler keeps these loads where
  // they are written instead of hoisting HW values an element out of the
  // step loop into registers (and scratch)
  auto load_op = [&](int q, R *h) {
    uint32_t off = (uint32_t)(tid + q * bs);
    asm volatile("" : "+v"(off));
    const R *hp = Hb + th.estart + off;
#pragma unroll
    for (int c = 0; c < HW; c++) h[c] = hp[(int64_t)c * a.Eexp];
  };
  // (halo: the element runs after the halo wait)
  auto element = [&](int q, bool halo) {
    const int64_t e = (int64_t)th.estart + tid + q * bs;
    const KLaw<R> kle = elem_law<GEN>(a, kl, e);
    if constexpr (OP != 0) {
      // the operator from registers, LDS or memory, then the element's load
      uint32_t off = (uint32_t)(tid + q * bs);
      asm volatile("" : "+v"(off));
      R h[HW];
      if (OPH && halo && r.ophalo) {
        const R *lp = oph + (off - (uint32_t)nint) * HWS;
#pragma unroll
        for (int c = 0; c < HW; c++) h[c] = lp[c];
      } else {
        load_op(q, h);
      }
      keep_packed(ew[q]);
      element_to_slots<R, NE, TDK, OP, NM>(ew[q], h, Tl, slot, nown, nown, a.pb, pmask, kle);
    } else if constexpr (PRE) {
      R T[8], V[8], F[8];
#pragma unroll
      for (int n = 0; n < 8; n++) T[n] = lds_ld<R>(ta[q][n]);
      if (tabs)
#pragma unroll
        for (int n = 0; n < 8; n++) V[n] = lds_ld<R>(ta[q][n] + dnv);
      Elem<R, 8>::load_vals(T, V, tabs, kle, TDK, eh[q], F);
#pragma unroll
      for (int n = 0; n < 8; n++) lds_st<R>(sa[q][n], F[n]);
    } else {
      keep_packed(ew[q]);
      element_to_slots<R, NE, TDK, 0, NM>(ew[q], eh[q], Tl, slot, nown, nown, a.pb, pmask, kle);
    }
  };
  // health: the step count of the first check that found a temperature of
  // the wave's nodes outside the window (wave-uniform, so it lives in a
  // scalar register), and the extremes since the last check (FP32, compared
  // with the window rounded outward); the energy check runs in the one-step
  // kernel
  int bad = -1;
  float tmn = INFINITY, tmx = -INFINITY;
  const float wlo = a.win_lo_f, whi = a.win_hi_f;
  // every load above completes here, once: otherwise the compiler waits for
  // them at their first use inside the loop, on every step, and such a wait
  // (vmcnt counts stores too) would also hold the interior elements until the
  // previous step's exports have completed
  __builtin_amdgcn_s_waitcnt(0x0f70);
  for (int s = 0; s < r.nsteps; s++) {
    // ---- stage the owned T from registers ----
#pragma unroll
    for (int q = 0; q < NPT; q++) {
      const int j = tid + q * bs;
      if (j < nown) {
        if constexpr (PRE) Tl[jpos[q]] = hi[q];
        else Tl[j] = hi[q];
        if (tabs) kl.stage(j, hi[q]);
      }
    }
    // ---- elements with every node owned need no halo value: they run while
    // the neighbours' exports of the previous step arrive (the barrier orders
    // them after the staging and after the previous step's slot sums) ----
    if (r.split) {
      __syncthreads();
#pragma unroll
      for (int q = 0; q < EPT; q++)
        if (tid + q * bs < nint) element(q, false);
    }
    // ---- halo from the state or the exchange, once the previous step's
    // export stores have completed (polling while they drain is slower;
    // s_waitcnt vmcnt(0)) ----
    __builtin_amdgcn_s_waitcnt(0x0f70);
    // a point-load schedule's row for this step: loaded now, its latency
    // hidden behind the halo wait, and put where the node phase reads the
    // record's power (each thread writes only the entries it reads itself)
    R pn[NPT];
    if (r.pts) {
      const R *rp = (const R *)r.pts + (int64_t)prow * r.pts_nrec + th.bstart;
#pragma unroll
      for (int q = 0; q < NPT; q++) {
        const int j = tid + q * bs;
        pn[q] = j < nbnd ? rp[j] : (R)0;
      }
      prow = prow + 1 == r.pts_nrows ? 0 : prow + 1;
    }
    R hv[HPT];
    if (s == 0) {
#pragma unroll
      for (int q = 0; q < HPT; q++) hv[q] = tid + q * bs < nhalo ? Tin[hid[q]] : (R)0;
    } else {
      const unsigned long long *X = r.X[s & 1];
      const unsigned want = r.tag0 + (unsigned)s + r.tag_skew;
      wait_halo<R, HPT>(X, hid, nhalo - tid, bs, want, hv, r.spin_limit, r.err);
    }
#pragma unroll
    for (int q = 0; q < HPT; q++) {
      const int j = tid + q * bs;
      if (j < nhalo) {
        if constexpr (PRE) Tl[hpos[q]] = hv[q];
        else Tl[nown + j] = hv[q];
        if (tabs) kl.stage(nown + j, hv[q]);
      }
    }
    if (r.pts) {
#pragma unroll
      for (int q = 0; q < NPT; q++) {
        const int j = tid + q * bs;
        if (j < nbnd) Lbnd[4 * nbnd + j] = pn[q];
      }
    }
    __syncthreads();
    // ---- the elements that touch the halo ----
#pragma unroll
    for (int q = 0; q < EPT; q++) {
      const int i = tid + q * bs;
      if (i >= nint && i < nE) element(q, true);
    }
    __syncthreads();
    // ---- per node: ordered sum, surface loads, explicit update, export ----
    // (the next step's owned staging writes only Tl, which nothing reads after
    // the barrier above; its slot writes come after a barrier, its halo writes
    // after the elements with every node owned, which read only owned T)
    unsigned long long *Xw = r.X[(s + 1) & 1];
    const unsigned tag = r.tag0 + (unsigned)s + 1u;
#pragma unroll
    for (int q = 0; q < NPT; q++) {
      const int j = tid + q * bs;
      if (j < nown) {
        const R F = NM ? slot_sum(slot + (PRE ? jpos[q] : j) * ((1 << a.pb) + 1), 0, 1, a.maxinc)
                       : slot_sum(slot, j, nown, a.maxinc);
        Node1<R> d;
        d.alpha = al[q];
        d.beta = be[q];
        d.lo = lo[q];
        const bool bnd = j < nbnd;
        if (bnd) {
          d.bA = Lbnd[j];
          d.bAT = Lbnd[nbnd + j];
          d.beA = Lbnd[2 * nbnd + j];
          d.bTa = Lbnd[3 * nbnd + j];
          d.bP = Lbnd[4 * nbnd + j];
        }
        float lo_new;
        R Q, den;
        hi[q] = advance<R, MODE, TDC>(d, bnd, hi[q], F, Tz, GEN ? (const R *)a.ctab : nullptr,
                                      GEN ? a.nct : 0, lo_new, Q, den);
        lo[q] = lo_new;
        if (ex[q]) Words<R>::put(Xw, th.nstart + j, tag, hi[q]);
        if (r.seg) ((R *)r.seg)[(int64_t)(s + 1) * r.segN + th.nstart + j] = hi[q];
      }
    }
    // ---- health: running extremes of the owned temperatures (after the
    // exports, off the neighbours' critical path), compared with the window
    // every kResCheck steps and at the launch's last step ----
#pragma unroll
    for (int q = 0; q < NPT; q++)
      if (tid + q * bs < nown) {
        tmn = fminf(tmn, (float)hi[q]);
        tmx = fmaxf(tmx, (float)hi[q]);
      }
    if ((s + 1) % kResCheck == 0 || s + 1 == r.nsteps) {
      bool out = tmn < wlo || tmx > whi;
#pragma unroll
      for (int q = 0; q < NPT; q++)
        if (tid + q * bs < nown) out = out || !(hi[q] == hi[q]);  // not a number
      if (bad < 0 && __ballot(out)) bad = s + 1;
      tmn = INFINITY;
      tmx = -INFINITY;
    }
  }
  // ---- final state of the owned nodes ----
  R *Tf = (R *)r.Tfin;
#pragma unroll
  for (int q = 0; q < NPT; q++) {
    const int j = tid + q * bs;
    if (j < nown) {
      Tf[th.nstart + j] = hi[q];
      if (MODE == 1) r.lofin[th.nstart + j] = lo[q];
    }
  }
  if (a.hl && bad >= 0 && (tid & 63) == 0) health_bad(a, health_step0(a) + bad);
}

// Resident adjoint: one launch runs the adjoint steps n1-1 .. n0
// of a checkpoint segment on the tiles of the resident forward kernel.  A tile
// keeps its elements (entries, operator) and its owned nodes' lambda in
// registers, the FP64 derivative sums of the elements it owns in registers
// (FP32) or LDS (FP64), and the boundary sums and per touched node alpha, beta,
// 1/dt and T^{n+1} in LDS; T^n of every node comes from the segment's stored
// states.  The halo's lambda^{n+1} travels as
// in the forward kernel: from the input at the first step, then through the
// tagged exchange words (the tiles and their neighbour relation are the
// forward's).  The arithmetic is that of k_adjoint1, so both give
// bitwise-identical multipliers and derivatives.
template <typename R, int MODE, bool GEN>
__global__ __launch_bounds__(1024) void k_adjres(AdjArgs a, AdjResArgs r) {
  constexpr int NE = 8;
  constexpr int EPT = ResCap<R, NE>::EPT, NPT = ResCap<R, NE>::NPT, HPT = ResCap<R, NE>::HPT;
  constexpr bool GREG = sizeof(R) == 4;  // derivative sums in registers, else LDS
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int b = blockIdx.x;
  const int t = (b & 7) * a.nper + (b >> 3);
  if (t >= a.nt) return;  // no tile: nobody reads from it
  const TileHdr th = a.tiles[t];
  const int nE = a.tiles[t].cum_e[0];
  const int nhalo = a.tiles[t].cum_n[1] - th.nown;
  const int tid = threadIdx.x, bs = blockDim.x;
  const int nown = th.nown, ntouch = nown + nhalo, nbnd = th.nbnd;
  const bool tdk = a.tdk != 0, tdc = a.tdc != 0;
  // LDS: FP64 boundary sums S0, S1 of the owned boundary nodes and (FP64
  // steps) the owners' derivative sums and rho V / n_e; then mu, w, T^n and T^{n+1} (two
  // buffers that swap every step), alpha, 1/dt (and beta) of the touched
  // nodes; the slots of the owned nodes; hA and sigma eps A of the owned
  // boundary nodes
  double *LS0 = reinterpret_cast<double *>(smem_raw);
  double *LS1 = LS0 + nbnd;
  double *Lgk = LS1 + nbnd;
  double *Lgc = Lgk + (GREG ? 0 : nE);
  R *Lmv = reinterpret_cast<R *>(Lgc + (GREG ? 0 : nE));  // FP64: rho V / n_e of the owners
  R *Lmu = Lmv + (GREG ? 0 : nE);
  R *Lw = Lmu + ntouch;
  R *LTa = Lw + ntouch;
  R *LTb = LTa + ntouch;
  R *Lal = LTb + ntouch;
  R *Lrdt = Lal + ntouch;
  R *Lbe = Lrdt + ntouch;  // tdc only
  R *slot = Lbe + (tdc ? ntouch : 0);  // node-major, every touched node (as in k_resident)
  const int sstride = (1 << a.pb) + 1, nslot = ntouch * sstride;
  R *LrA = slot + nslot;
  R *LreA = LrA + nbnd;
  const R *ctab = GEN ? (const R *)a.ctab : nullptr;
  const int nct = GEN ? a.nct : 0;
  using EntT = typename Ent<NE>::T;
  const EntT *ent = reinterpret_cast<const EntT *>(a.ent);
  const R *Hb = (const R *)a.H;
  EntT ew[EPT];
  R eh[EPT][6], emv[GREG ? EPT : 1];
  double gk[GREG ? EPT : 1], gc[GREG ? EPT : 1];
  uint32_t own = 0;
#pragma unroll
  for (int q = 0; q < EPT; q++) {
    const int i = tid + q * bs;
    if (GREG) {
      gk[q] = gc[q] = 0.0;
      emv[q] = (R)0;
    }
    if (i < nE) {
      const int64_t e = (int64_t)th.estart + i;
      ew[q] = ent[e];
#pragma unroll
      for (int c = 0; c < 6; c++) eh[q][c] = Hb[(int64_t)c * a.Eexp + e];
      if (a.eowner[e]) {
        const int32_t eo = a.eorig[e];
        own |= 1u << q;
        if (GREG) {
          gk[q] = a.g_logk[eo];
          gc[q] = a.g_c[eo];
          emv[q] = ((const R *)a.mV)[eo];
        } else {
          Lgk[i] = a.g_logk[eo];
          Lgc[i] = a.g_c[eo];
          Lmv[i] = ((const R *)a.mV)[eo];
        }
      }
    }
  }
  const R *lamin = (const R *)a.lamin;
  R lam[NPT];
  float llo[NPT];
  bool ex[NPT];
#pragma unroll
  for (int q = 0; q < NPT; q++) {
    const int j = tid + q * bs;
    ex[q] = false;
    if (j < nown) {
      const int k = th.nstart + j;
      lam[q] = lamin[k];
      llo[q] = MODE == 1 ? a.lamloin[k] : 0.0f;
      ex[q] = r.exported[k] != 0;
    }
  }
  int hid[HPT];
#pragma unroll
  for (int q = 0; q < HPT; q++) {
    const int j = tid + q * bs;
    hid[q] = j < nhalo ? a.halo[th.hstart + j] : 0;
  }
  const R *segT = (const R *)r.seg;
  {
    const R *Tlast = segT + (int64_t)r.nsteps * r.segN;  // T^{n1}
    for (int j = tid; j < ntouch; j += bs) {
      const int g = j < nown ? th.nstart + j : a.halo[th.hstart + j - nown];
      Lal[j] = ((const R *)a.alpha)[g];
      Lrdt[j] = ((const R *)a.rdt)[g];
      if (tdc) Lbe[j] = ((const R *)a.beta)[g];
      LTb[j] = Tlast[g];
    }
    for (int j = tid; j < nbnd; j += bs) {
      LrA[j] = ((const R *)a.rA)[th.bstart + j];
      LreA[j] = ((const R *)a.reA)[th.bstart + j];
      LS0[j] = a.S0[th.bstart + j];
      LS1[j] = a.S1[th.bstart + j];
    }
    // slots past a node's incidence are never written and stay zero
    for (int j = tid; j < nslot; j += bs) slot[j] = (R)0;
  }
  __syncthreads();
  const KLaw<R> kl = GEN ? KLaw<R>{(R)a.s0, (R)a.s1, (const R *)a.ktab, a.nkt}
                         : KLaw<R>{(R)a.s0, (R)a.s1, nullptr, 0};
  const R Tz = (R)a.Tz;
  const uint32_t pmask = (1u << a.pb) - 1u;
  R *LT = LTa, *LTp = LTb;  // T^n, T^{n+1}
  for (int s = 0; s < r.nsteps; s++) {
    __builtin_amdgcn_s_waitcnt(0x0f70);  // as in k_resident
    const R *Ti = segT + (int64_t)(r.nsteps - 1 - s) * r.segN;  // T^n, n = n1 - 1 - s
    // ---- T^n of the touched nodes (stored states) ----
    R tno[NPT], tnh[HPT];
#pragma unroll
    for (int q = 0; q < NPT; q++) tno[q] = tid + q * bs < nown ? Ti[th.nstart + tid + q * bs] : (R)0;
#pragma unroll
    for (int q = 0; q < HPT; q++) tnh[q] = tid + q * bs < nhalo ? Ti[hid[q]] : (R)0;
    // ---- lambda^{n+1} of the halo: the input, or the exchange ----
    R hv[HPT];
    if (s == 0) {
#pragma unroll
      for (int q = 0; q < HPT; q++) hv[q] = tid + q * bs < nhalo ? lamin[hid[q]] : (R)0;
    } else {
      const unsigned long long *X = r.X[s & 1];
      const unsigned want = r.tag0 + (unsigned)s;
      wait_halo<R, HPT>(X, hid, nhalo - tid, bs, want, hv, r.spin_limit, r.err);
    }
    // ---- stage mu, w, T^n (owned by their node's thread, halo by the halo thread) ----
#pragma unroll
    for (int q = 0; q < NPT; q++) {
      const int j = tid + q * bs;
      if (j < nown) {
        adj_stage<R>(lam[q], Lal[j], tdc ? Lbe[j] : (R)0, tno[q], LTp[j], Lrdt[j], tdc, ctab, nct,
                     Lmu[j], Lw[j]);
        LT[j] = tno[q];
      }
    }
#pragma unroll
    for (int q = 0; q < HPT; q++) {
      const int j = nown + tid + q * bs;
      if (j < ntouch) {
        adj_stage<R>(hv[q], Lal[j], tdc ? Lbe[j] : (R)0, tnh[q], LTp[j], Lrdt[j], tdc, ctab, nct,
                     Lmu[j], Lw[j]);
        LT[j] = tnh[q];
      }
    }
    __syncthreads();
    // ---- elements: slots, and the owners' derivative sums ----
#pragma unroll
    for (int q = 0; q < EPT; q++)
      if (tid + q * bs < nE) {
        keep_packed(ew[q]);
        uint32_t v[NE], loc[NE];
        Ent<NE>::unpack(ew[q], v);
#pragma unroll
        for (int n = 0; n < NE; n++) loc[n] = v[n] >> a.pb;
        const bool owner = (own >> q) & 1u;
        R F[NE], se, muKT, gsum;
        adj_elem<R, NE, 0>(loc, eh[q], kl, tdk, owner, Lmu, LT, Lw, F, se, muKT, gsum);
#pragma unroll
        for (int n = 0; n < NE; n++) slot[v[n] + loc[n]] = F[n];
        if (owner) {
          if (GREG) adj_grad<R>(gk[q], gc[q], se, muKT, emv[q], gsum);
          else adj_grad<R>(Lgk[tid + q * bs], Lgc[tid + q * bs], se, muKT, Lmv[tid + q * bs], gsum);
        }
      }
    __syncthreads();
    // ---- owned nodes: lambda^n, boundary sums, export ----
    // (the next staging rewrites only entries its own thread reads here)
    unsigned long long *Xw = r.X[(s + 1) & 1];
    const unsigned tag = r.tag0 + (unsigned)s + 1u;
#pragma unroll
    for (int q = 0; q < NPT; q++) {
      const int j = tid + q * bs;
      if (j < nown) {
        const R F = slot_sum(slot + j * sstride, 0, 1, a.maxinc);
        const R mu = Lmu[j], tn = LT[j], tn1 = LTp[j], al = Lal[j];
        const bool bnd = j < nbnd;
        const R dden = tdc ? adj_dden<R>(al, Lbe[j], tn, ctab, nct) : (R)0;
        const R d = adj_node<R>(F, mu, bnd, bnd ? LrA[j] : (R)0, bnd ? LreA[j] : (R)0, tn, tn1, Tz,
                                tdc, dden);
        if (bnd) adj_bnd<R>(LS0[j], LS1[j], mu, tn);
        float lo_new;
        lam[q] = adj_lambda<R, MODE>(lam[q], llo[q], d, al == (R)INFINITY, lo_new);
        llo[q] = lo_new;
        if (ex[q]) Words<R>::put(Xw, th.nstart + j, tag, lam[q]);
      }
    }
    R *tmp = LT;
    LT = LTp;
    LTp = tmp;
  }
  // ---- results: lambda^{n0}, the boundary sums, the owners' derivative sums ----
  R *lout = (R *)a.lamout;
#pragma unroll
  for (int q = 0; q < NPT; q++) {
    const int j = tid + q * bs;
    if (j < nown) {
      lout[th.nstart + j] = lam[q];
      if (MODE == 1) a.lamloout[th.nstart + j] = llo[q];
      if (j < nbnd) {
        a.S0[th.bstart + j] = LS0[j];
        a.S1[th.bstart + j] = LS1[j];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < EPT; q++)
    if ((own >> q) & 1u) {
      const int i = tid + q * bs;
      const int32_t eo = a.eorig[(int64_t)th.estart + i];
      a.g_logk[eo] = GREG ? gk[q] : Lgk[i];
      a.g_c[eo] = GREG ? gc[q] : Lgc[i];
    }
}

}  // namespace

// ---------------------------------------------------------------------------
hipError_t launch_geom(const GeomArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_geom, dim3(blocks_for(a.E, 128)), dim3(128), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_mass(const MassArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_mass, dim3(blocks_for(a.N, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_bnd(const BndArgs &a, hipStream_t s) {
  if (a.nf > 0) hipLaunchKernelGGL(k_face_area, dim3(blocks_for(a.nf, 256)), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (a.nrec > 0) hipLaunchKernelGGL(k_bnd_rec, dim3(blocks_for(a.nrec, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_point_rows(int prec, const BndArgs &a, int64_t nrows, int64_t npt,
                             const double *W, void *out, hipStream_t s) {
  const int64_t n = nrows * a.nrec;
  if (n == 0) return hipSuccess;
  if (prec == 1)
    hipLaunchKernelGGL(k_point_rows<double>, dim3(blocks_for(n, 256)), dim3(256), 0, s, a, nrows,
                       npt, W, (double *)out);
  else
    hipLaunchKernelGGL(k_point_rows<float>, dim3(blocks_for(n, 256)), dim3(256), 0, s, a, nrows,
                       npt, W, (float *)out);
  return hipGetLastError();
}

hipError_t launch_dt(const DtArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_dt_elem, dim3(blocks_for(a.E, 256)), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (a.nrec > 0) hipLaunchKernelGGL(k_dt_node, dim3(blocks_for(a.nrec, 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_node_arrays(const NodeArrArgs &a, hipStream_t s) {
  int64_t n = a.N > a.nrec ? a.N : a.nrec;
  if (a.prec == 1)
    hipLaunchKernelGGL(k_node_arrays<double>, dim3(blocks_for(n, 256)), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_node_arrays<float>, dim3(blocks_for(n, 256)), dim3(256), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return hipSuccess;
}

hipError_t launch_expand_sk(int prec, int64_t Eexp, const int32_t *eorig, const MatDev *mats,
                            const int32_t *emat, void *esk, hipStream_t s) {
  if (prec == 1)
    hipLaunchKernelGGL(k_expand_sk<double>, dim3(blocks_for(Eexp, 256)), dim3(256), 0, s, Eexp,
                       eorig, mats, emat, (double *)esk);
  else
    hipLaunchKernelGGL(k_expand_sk<float>, dim3(blocks_for(Eexp, 256)), dim3(256), 0, s, Eexp,
                       eorig, mats, emat, (float *)esk);
  return hipGetLastError();
}

hipError_t launch_expand_H(int prec, int W, int from, int to, int64_t Eexp, int64_t E, const int32_t *eorig,
                           const double *H0, const double *kscale, void *H, hipStream_t s) {
  if (prec == 1)
    hipLaunchKernelGGL(k_expand_H<double>, dim3(blocks_for(Eexp, 256)), dim3(256), 0, s, W, from,
                       to, Eexp, E, eorig, H0, kscale, (double *)H);
  else
    hipLaunchKernelGGL(k_expand_H<float>, dim3(blocks_for(Eexp, 256)), dim3(256), 0, s, W, from,
                       to, Eexp, E, eorig, H0, kscale, (float *)H);
  return hipGetLastError();
}

hipError_t launch_step(const StepArgs &a, hipStream_t s) {
  if (a.prec == 1)
    return a.ne == 8 ? step_dispatch_tt<double, 8, 0>(a, s) : step_dispatch_tt<double, 4, 0>(a, s);
  if (a.prec == 0)
    return a.ne == 8 ? step_dispatch_tt<float, 8, 1>(a, s) : step_dispatch_tt<float, 4, 1>(a, s);
  return a.ne == 8 ? step_dispatch_tt<float, 8, 0>(a, s) : step_dispatch_tt<float, 4, 0>(a, s);
}

hipError_t step_set_lds_limit(int prec, int ne, int tdk, int tdc, int gen, int op, int bytes) {
  if (prec == 1)
    return ne == 8 ? attr_dispatch_tt<double, 8, 0>(tdk, tdc, gen, op, bytes) : attr_dispatch_tt<double, 4, 0>(tdk, tdc, gen, op, bytes);
  if (prec == 0)
    return ne == 8 ? attr_dispatch_tt<float, 8, 1>(tdk, tdc, gen, op, bytes) : attr_dispatch_tt<float, 4, 1>(tdk, tdc, gen, op, bytes);
  return ne == 8 ? attr_dispatch_tt<float, 8, 0>(tdk, tdc, gen, op, bytes) : attr_dispatch_tt<float, 4, 0>(tdk, tdc, gen, op, bytes);
}

hipError_t launch_set_T(int prec, int64_t N, const double *Tuser, const int32_t *perm, void *T,
                        float *lo, int64_t ndir, const int32_t *dir_node, const double *dir_T,
                        hipStream_t s) {
  dim3 g(blocks_for(N, 256)), gd(blocks_for(ndir, 256)), b(256);
  if (prec == 1) {
    hipLaunchKernelGGL((k_set_T<double, 0>), g, b, 0, s, N, Tuser, perm, (double *)T, lo);
    if (ndir) hipLaunchKernelGGL((k_set_dir<double, 0>), gd, b, 0, s, ndir, dir_node, dir_T, (double *)T, lo);
  } else if (prec == 0) {
    hipLaunchKernelGGL((k_set_T<float, 1>), g, b, 0, s, N, Tuser, perm, (float *)T, lo);
    if (ndir) hipLaunchKernelGGL((k_set_dir<float, 1>), gd, b, 0, s, ndir, dir_node, dir_T, (float *)T, lo);
  } else {
    hipLaunchKernelGGL((k_set_T<float, 0>), g, b, 0, s, N, Tuser, perm, (float *)T, lo);
    if (ndir) hipLaunchKernelGGL((k_set_dir<float, 0>), gd, b, 0, s, ndir, dir_node, dir_T, (float *)T, lo);
  }
  return hipGetLastError();
}

hipError_t launch_get_T(int prec, int64_t N, const int32_t *perm, const void *T, const float *lo,
                        double *Tuser, hipStream_t s) {
  dim3 g(blocks_for(N, 256)), b(256);
  if (prec == 1)
    hipLaunchKernelGGL((k_get_T<double, 0>), g, b, 0, s, N, perm, (const double *)T, lo, Tuser);
  else if (prec == 0)
    hipLaunchKernelGGL((k_get_T<float, 1>), g, b, 0, s, N, perm, (const float *)T, lo, Tuser);
  else
    hipLaunchKernelGGL((k_get_T<float, 0>), g, b, 0, s, N, perm, (const float *)T, lo, Tuser);
  return hipGetLastError();
}

hipError_t launch_check(int prec, int64_t N, const void *T, const float *lo, double lo_b,
                        double hi_b, int *flag, hipStream_t s) {
  dim3 g(blocks_for(N, 256)), b(256);
  if (prec == 1)
    hipLaunchKernelGGL((k_check<double, 0>), g, b, 0, s, N, (const double *)T, lo, lo_b, hi_b, flag);
  else if (prec == 0)
    hipLaunchKernelGGL((k_check<float, 1>), g, b, 0, s, N, (const float *)T, lo, lo_b, hi_b, flag);
  else
    hipLaunchKernelGGL((k_check<float, 0>), g, b, 0, s, N, (const float *)T, lo, lo_b, hi_b, flag);
  return hipGetLastError();
}

hipError_t launch_health(Health *h, int op, long long v, hipStream_t s) {
  hipLaunchKernelGGL(k_health, dim3(1), dim3(1), 0, s, h, op, v);
  return hipGetLastError();
}

hipError_t launch_range(int prec, int64_t N, const void *T, const float *lo,
                        unsigned long long *keys, int *nan, hipStream_t s) {
  dim3 g(blocks_for(N, 256)), b(256);
  if (prec == 1)
    hipLaunchKernelGGL((k_range<double, 0>), g, b, 0, s, N, (const double *)T, lo, keys, nan);
  else if (prec == 0)
    hipLaunchKernelGGL((k_range<float, 1>), g, b, 0, s, N, (const float *)T, lo, keys, nan);
  else
    hipLaunchKernelGGL((k_range<float, 0>), g, b, 0, s, N, (const float *)T, lo, keys, nan);
  return hipGetLastError();
}

hipError_t launch_permute(int elem_bytes, int64_t N, const int32_t *perm, const void *src,
                          void *dst, int to_internal, hipStream_t s) {
  hipLaunchKernelGGL(k_permute, dim3(blocks_for(N, 256)), dim3(256), 0, s, elem_bytes, N, perm,
                     (const unsigned char *)src, (unsigned char *)dst, to_internal);
  return hipGetLastError();
}

}  // namespace fed

namespace fed {

template <typename R, int NE, int MODE, bool TDK, bool TDC, bool GEN, int OP = 0>
const void *resident_fn() {
  return (const void *)k_resident<R, NE, MODE, TDK, TDC, GEN, OP>;
}

// tables and per-element laws run the general instance, and so does the
// uniform-gradient hexahedron (op 1, 2)
template <typename R, int NE, int MODE>
const void *resident_tt(int tdk, int tdc, bool gen, int op) {
  // (the linear laws' instance with both laws on: a law with zero slope gives
  // the same bits, fma(0, T, s0) = s0)
  if (NE == 8 && op == 1)
    return gen ? resident_fn<R, 8, MODE, true, true, true, 1>()
               : resident_fn<R, 8, MODE, true, true, false, 1>();
  if (NE == 8 && op == 2)
    return gen ? resident_fn<R, 8, MODE, true, true, true, 2>()
               : resident_fn<R, 8, MODE, true, true, false, 2>();
  if (gen) return resident_fn<R, NE, MODE, true, true, true>();
  if (tdk)
    return tdc ? resident_fn<R, NE, MODE, true, true, false>() : resident_fn<R, NE, MODE, true, false, false>();
  return tdc ? resident_fn<R, NE, MODE, false, true, false>() : resident_fn<R, NE, MODE, false, false, false>();
}

const void *resident_kernel(const StepArgs &a) {
  const bool g = a.ktab || a.ctab || a.esk;
  if (a.prec == 1)
    return a.ne == 8 ? resident_tt<double, 8, 0>(a.tdk, a.tdc, g, a.op)
                     : resident_tt<double, 4, 0>(a.tdk, a.tdc, g, 0);
  if (a.prec == 0)
    return a.ne == 8 ? resident_tt<float, 8, 1>(a.tdk, a.tdc, g, a.op)
                     : resident_tt<float, 4, 1>(a.tdk, a.tdc, g, 0);
  return a.ne == 8 ? resident_tt<float, 8, 0>(a.tdk, a.tdc, g, a.op)
                   : resident_tt<float, 4, 0>(a.tdk, a.tdc, g, 0);
}

ResCaps resident_caps(int prec, int ne) {
  if (prec == 1)
    return ne == 8 ? ResCaps{ResCap<double, 8>::EPT, ResCap<double, 8>::NPT, ResCap<double, 8>::HPT}
                   : ResCaps{ResCap<double, 4>::EPT, ResCap<double, 4>::NPT, ResCap<double, 4>::HPT};
  return ne == 8 ? ResCaps{ResCap<float, 8>::EPT, ResCap<float, 8>::NPT, ResCap<float, 8>::HPT}
                 : ResCaps{ResCap<float, 4>::EPT, ResCap<float, 4>::NPT, ResCap<float, 4>::HPT};
}

hipError_t resident_prepare(const StepArgs &a, int *blocks_per_cu) {
  const void *f = resident_kernel(a);
  hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, a.lds);
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, f, a.block, a.lds);
}

// Resident launches are ordinary launches: the grid fits the workgroups the
// GPU holds at once (checked when the context is made, with the occupancy of
// resident_prepare), so on a GPU that runs nothing else every tile is resident
// from the start.  A cooperative launch guarantees the same but costs about
// 14 us more per launch (it waits for the device); if another stream's
// kernels hold CUs, tiles not yet resident start once those finish, and the
// bounded halo waits (seconds) end a launch that cannot proceed with an
// error instead of a hang.
hipError_t launch_resident(const StepArgs &a, const ResArgs &r, hipStream_t s) {
  StepArgs aa = a;
  ResArgs rr = r;
  void *args[] = {(void *)&aa, (void *)&rr};
  return hipLaunchKernel(resident_kernel(a), dim3(8 * a.nper), dim3(a.block), args,
                         (size_t)a.lds, s);
}

const void *adjres_kernel(int prec, bool gen) {
  if (gen) {
    if (prec == 1) return (const void *)k_adjres<double, 0, true>;
    if (prec == 0) return (const void *)k_adjres<float, 1, true>;
    return (const void *)k_adjres<float, 0, true>;
  }
  if (prec == 1) return (const void *)k_adjres<double, 0, false>;
  if (prec == 0) return (const void *)k_adjres<float, 1, false>;
  return (const void *)k_adjres<float, 0, false>;
}

hipError_t adjres_prepare(int prec, int gen, int block, int lds, int *blocks_per_cu) {
  const void *f = adjres_kernel(prec, gen != 0);
  hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return e;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, f, block, lds);
}

hipError_t launch_adjres(const AdjArgs &a, const AdjResArgs &r, hipStream_t s) {
  AdjArgs aa = a;
  AdjResArgs rr = r;
  void *args[] = {(void *)&aa, (void *)&rr};
  // an ordinary launch, as launch_resident
  return hipLaunchKernel(adjres_kernel(a.prec, a.ktab || a.ctab || a.esk), dim3(8 * a.nper),
                         dim3(a.block), args, (size_t)a.lds, s);
}

// the one-step adjoint instance of (precision, element, operator, laws)
template <bool GEN>
const void *adjoint_kernel_t(int prec, int ne, int op) {
  if (ne == 8 && op == 1)
    return prec == 1 ? (const void *)k_adjoint1<double, 8, 0, 1, GEN>
                     : (prec == 0 ? (const void *)k_adjoint1<float, 8, 1, 1, GEN>
                                  : (const void *)k_adjoint1<float, 8, 0, 1, GEN>);
  if (ne == 8 && op == 2)
    return prec == 1 ? (const void *)k_adjoint1<double, 8, 0, 2, GEN>
                     : (prec == 0 ? (const void *)k_adjoint1<float, 8, 1, 2, GEN>
                                  : (const void *)k_adjoint1<float, 8, 0, 2, GEN>);
  if (prec == 1)
    return ne == 8 ? (const void *)k_adjoint1<double, 8, 0, 0, GEN>
                   : (const void *)k_adjoint1<double, 4, 0, 0, GEN>;
  if (prec == 0)
    return ne == 8 ? (const void *)k_adjoint1<float, 8, 1, 0, GEN>
                   : (const void *)k_adjoint1<float, 4, 1, 0, GEN>;
  return ne == 8 ? (const void *)k_adjoint1<float, 8, 0, 0, GEN>
                 : (const void *)k_adjoint1<float, 4, 0, 0, GEN>;
}

const void *adjoint_kernel(int prec, int ne, int op, bool gen) {
  return gen ? adjoint_kernel_t<true>(prec, ne, op) : adjoint_kernel_t<false>(prec, ne, op);
}

hipError_t launch_adjoint(const AdjArgs &a, hipStream_t s) {
  AdjArgs aa = a;
  void *args[] = {(void *)&aa};
  return hipLaunchKernel(adjoint_kernel(a.prec, a.ne, a.op, a.ktab || a.ctab || a.esk),
                         dim3(8 * a.nper), dim3(a.block), args, (size_t)a.lds, s);
}

hipError_t adjoint_set_lds_limit(int prec, int ne, int op, int bytes) {
  for (int g = 0; g < 2; g++) {
    hipError_t e = hipFuncSetAttribute(adjoint_kernel(prec, ne, op, g != 0),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_face_grad(int64_t nf, int nfn, const int32_t *faces, const int32_t *perm,
                            const int32_t *rec_of, const double *farea, const double *fTa,
                            const double *S0, const double *S1, double *g_h, hipStream_t s) {
  if (nf == 0) return hipSuccess;
  hipLaunchKernelGGL(k_face_grad, dim3(blocks_for(nf, 256)), dim3(256), 0, s, nf, nfn, faces,
                     perm, rec_of, farea, fTa, S0, S1, g_h);
  return hipGetLastError();
}

hipError_t launch_adjoint_coefs(int prec, int64_t N, int64_t E, int ne, const double *dt_inst,
                                const int32_t *node_inst, const MatDev *mats,
                                const int32_t *emat, const double *V, void *rdt, void *mV,
                                hipStream_t s) {
  int64_t n = N > E ? N : E;
  if (prec == 1)
    hipLaunchKernelGGL(k_adjoint_coefs<double>, dim3(blocks_for(n, 256)), dim3(256), 0, s, N, E,
                       ne, dt_inst, node_inst, mats, emat, V, (double *)rdt, (double *)mV);
  else
    hipLaunchKernelGGL(k_adjoint_coefs<float>, dim3(blocks_for(n, 256)), dim3(256), 0, s, N, E,
                       ne, dt_inst, node_inst, mats, emat, V, (float *)rdt, (float *)mV);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free adjoint entry point: one array in the code
// object, which every GPU the library runs on holds until the process ends.
// Host code never uses the array's name as an address (on the host it names
// a stand-in, not device memory): scratch_address looks the device address up
// once per device, with that device current, and every kernel argument,
// memset and copy uses that address.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_address(void **ptr) {
  static std::mutex mu;
  static std::vector<void *> addr;  // per device
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
  if (!addr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

}  // namespace fed
