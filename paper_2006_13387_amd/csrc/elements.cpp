// Element matrices of the bilinear (Q1) square element, evaluated on the
// host by 2 x 2 Gauss quadrature (exact for these polynomial integrands),
// and the stiffness of the trilinear (H8) brick.
//
// Paper Section 1.1: C = E(x) C0 with C0 the plane-stress tensor of unit
// modulus; the stiffness of element e is E_e times the unit-modulus matrix.
// Section 4.1: the heat eigenproblem uses the scalar stiffness and mass.
//
// Vertex a = ax + 2*ay of the element [0,h]^2; DOF 2a + c.
#include <cmath>

namespace msp {

static void shape_q1(double xi, double eta, double N[4], double dNx[4],
                     double dNy[4]) {
  for (int a = 0; a < 4; ++a) {
    const int ax = a & 1, ay = a >> 1;
    const double fx = ax ? xi : 1.0 - xi, fy = ay ? eta : 1.0 - eta;
    const double gx = ax ? 1.0 : -1.0, gy = ay ? 1.0 : -1.0;
    N[a] = fx * fy;
    dNx[a] = gx * fy;
    dNy[a] = fx * gy;
  }
}

// Ke[8*8]: unit-modulus plane-stress stiffness; Ae, Me [4*4]: scalar
// stiffness and consistent mass (unit coefficient).
void q1_element_matrices(double nu, double h, double* Ke, double* Ae,
                         double* Me) {
  const double g = 0.5 / std::sqrt(3.0);
  const double pts[2] = {0.5 - g, 0.5 + g};
  const double c = 1.0 / (1.0 - nu * nu);
  const double D[3][3] = {{c, c * nu, 0.0}, {c * nu, c, 0.0},
                          {0.0, 0.0, c * 0.5 * (1.0 - nu)}};
  for (int i = 0; i < 64; ++i) Ke[i] = 0.0;
  for (int i = 0; i < 16; ++i) Ae[i] = Me[i] = 0.0;
  for (int qx = 0; qx < 2; ++qx)
    for (int qy = 0; qy < 2; ++qy) {
      double N[4], dx[4], dy[4];
      shape_q1(pts[qx], pts[qy], N, dx, dy);
      const double w = 0.25 * h * h;           // weight * |J|
      for (int a = 0; a < 4; ++a) {
        dx[a] /= h;
        dy[a] /= h;
      }
      double B[3][8] = {};
      for (int a = 0; a < 4; ++a) {
        B[0][2 * a] = dx[a];
        B[1][2 * a + 1] = dy[a];
        B[2][2 * a] = dy[a];
        B[2][2 * a + 1] = dx[a];
      }
      for (int i = 0; i < 8; ++i)
        for (int j = 0; j < 8; ++j) {
          double s = 0.0;
          for (int p = 0; p < 3; ++p)
            for (int q = 0; q < 3; ++q) s += B[p][i] * D[p][q] * B[q][j];
          Ke[i * 8 + j] += w * s;
        }
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
          Ae[a * 4 + b] += w * (dx[a] * dx[b] + dy[a] * dy[b]);
          Me[a * 4 + b] += w * N[a] * N[b];
        }
    }
}

// Ke[24*24]: unit-modulus stiffness of the trilinear (H8) brick element of
// edge h by 2 x 2 x 2 Gauss quadrature (exact here), isotropic with the
// Lame constants of E = 1: lambda = nu / ((1 + nu)(1 - 2 nu)),
// mu = 1 / (2 (1 + nu)).  Vertex a = ax + 2 ay + 4 az, DOF 3a + c; strains
// in the order xx, yy, zz, xy, yz, zx with engineering shears.
void h8_element_stiffness(double nu, double h, double* Ke) {
  const double g = 0.5 / std::sqrt(3.0);
  const double pts[2] = {0.5 - g, 0.5 + g};
  const double lam = nu / ((1.0 + nu) * (1.0 - 2.0 * nu)), mu = 0.5 / (1.0 + nu);
  double D[6][6] = {};
  for (int p = 0; p < 3; ++p) {
    for (int q = 0; q < 3; ++q) D[p][q] = lam;
    D[p][p] = lam + 2.0 * mu;
    D[p + 3][p + 3] = mu;
  }
  for (int i = 0; i < 576; ++i) Ke[i] = 0.0;
  for (int qz = 0; qz < 2; ++qz)
    for (int qy = 0; qy < 2; ++qy)
      for (int qx = 0; qx < 2; ++qx) {
        const double xi[3] = {pts[qx], pts[qy], pts[qz]};
        double B[6][24] = {};
        for (int a = 0; a < 8; ++a) {
          const int bit[3] = {a & 1, (a >> 1) & 1, a >> 2};
          double f[3], dg[3];
          for (int d = 0; d < 3; ++d) {
            f[d] = bit[d] ? xi[d] : 1.0 - xi[d];
            dg[d] = bit[d] ? 1.0 : -1.0;
          }
          const double dx = dg[0] * f[1] * f[2] / h;
          const double dy = f[0] * dg[1] * f[2] / h;
          const double dz = f[0] * f[1] * dg[2] / h;
          B[0][3 * a] = dx;
          B[1][3 * a + 1] = dy;
          B[2][3 * a + 2] = dz;
          B[3][3 * a] = dy;
          B[3][3 * a + 1] = dx;
          B[4][3 * a + 1] = dz;
          B[4][3 * a + 2] = dy;
          B[5][3 * a] = dz;
          B[5][3 * a + 2] = dx;
        }
        const double w = 0.125 * h * h * h;     // weight * |J|
        for (int i = 0; i < 24; ++i)
          for (int j = 0; j < 24; ++j) {
            double s = 0.0;
            for (int p = 0; p < 6; ++p)
              for (int q = 0; q < 6; ++q) s += B[p][i] * D[p][q] * B[q][j];
            Ke[i * 24 + j] += w * s;
          }
      }
}


// Ae[8*8], Me[8*8]: scalar stiffness int grad N . grad N and consistent mass
// int N N of the trilinear brick of edge h (the 3D heat pencil of Section
// 4.1, unit coefficient).  Both are tensor products of the linear element's
// 1D matrices k1 = [1 -1; -1 1] / h and m1 = h [2 1; 1 2] / 6:
// Ae = k1 x m1 x m1 + m1 x k1 x m1 + m1 x m1 x k1, Me = m1 x m1 x m1.
void h8_heat_element(double h, double* Ae, double* Me) {
  const double k1[2][2] = {{1.0 / h, -1.0 / h}, {-1.0 / h, 1.0 / h}};
  const double m1[2][2] = {{h / 3.0, h / 6.0}, {h / 6.0, h / 3.0}};
  for (int a = 0; a < 8; ++a)
    for (int b = 0; b < 8; ++b) {
      const int ax = a & 1, ay = (a >> 1) & 1, az = a >> 2;
      const int bx = b & 1, by = (b >> 1) & 1, bz = b >> 2;
      Ae[a * 8 + b] = k1[ax][bx] * m1[ay][by] * m1[az][bz] +
                      m1[ax][bx] * k1[ay][by] * m1[az][bz] +
                      m1[ax][bx] * m1[ay][by] * k1[az][bz];
      Me[a * 8 + b] = m1[ax][bx] * m1[ay][by] * m1[az][bz];
    }
}

}  // namespace msp
