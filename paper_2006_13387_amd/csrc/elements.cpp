// Element matrices of the bilinear (Q1) square element, evaluated on the
// host by 2 x 2 Gauss quadrature (exact for these polynomial integrands).
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

}  // namespace msp
