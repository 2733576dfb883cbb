// Host helper: sample-frame stiffness and eigenstrain tables of Mg tension
// twins (Sec. 2.1 of the paper: c/a, the six {10-12}<-1011> variants and the
// twin stiffness (C_twin)_ijkl = C_abcd Q_ia Q_jb Q_kc Q_ld; Table 2: elastic
// constants; twin shear 0.129).
#include <cmath>
#include <cstring>

#include "../../include/pf.h"

namespace {

struct V3 {
  double v[3];
};

V3 cross(const V3& a, const V3& b) {
  return {{a.v[1] * b.v[2] - a.v[2] * b.v[1], a.v[2] * b.v[0] - a.v[0] * b.v[2], a.v[0] * b.v[1] - a.v[1] * b.v[0]}};
}
double dot(const V3& a, const V3& b) { return a.v[0] * b.v[0] + a.v[1] * b.v[1] + a.v[2] * b.v[2]; }
V3 axpy(double s, const V3& a, const V3& b) {
  return {{s * a.v[0] + b.v[0], s * a.v[1] + b.v[1], s * a.v[2] + b.v[2]}};
}
V3 unit(const V3& a) {
  const double n = std::sqrt(dot(a, a));
  return {{a.v[0] / n, a.v[1] / n, a.v[2] / n}};
}

// The six tension-twin variants: plane (h k i l) and direction [u v t w].
const int kVariants[6][2][4] = {
    {{1, 0, -1, 2}, {-1, 0, 1, 1}},  {{-1, 0, 1, 2}, {1, 0, -1, 1}},
    {{0, 1, -1, 2}, {0, -1, 1, 1}},  {{0, -1, 1, 2}, {0, 1, -1, 1}},
    {{1, -1, 0, 2}, {-1, 1, 0, 1}},  {{-1, 1, 0, 2}, {1, -1, 0, 1}},
};

// Voigt index of the tensor pair (i, j): xx yy zz yz xz xy.
int voigt(int i, int j) {
  static const int map[3][3] = {{0, 5, 4}, {5, 1, 3}, {4, 3, 2}};
  return map[i][j];
}

// C'_ijkl = R_ia R_jb R_kc R_ld C_abcd on 6x6 Voigt matrices (engineering
// convention; C_ijkl = Cv[voigt(i,j)][voigt(k,l)]).
void rotate_voigt(const double* Cv, const double R[3][3], double* out) {
  double C[3][3][3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) C[i][j][k][l] = Cv[6 * voigt(i, j) + voigt(k, l)];
  // contract one index at a time
  double T1[3][3][3][3], T2[3][3][3][3];
  for (int i = 0; i < 3; ++i)
    for (int b = 0; b < 3; ++b)
      for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) {
          double s = 0;
          for (int a = 0; a < 3; ++a) s += R[i][a] * C[a][b][c][d];
          T1[i][b][c][d] = s;
        }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) {
          double s = 0;
          for (int b = 0; b < 3; ++b) s += R[j][b] * T1[i][b][c][d];
          T2[i][j][c][d] = s;
        }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k)
        for (int d = 0; d < 3; ++d) {
          double s = 0;
          for (int c = 0; c < 3; ++c) s += R[k][c] * T2[i][j][c][d];
          T1[i][j][k][d] = s;
        }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) {
          double s = 0;
          for (int d = 0; d < 3; ++d) s += R[l][d] * T1[i][j][k][d];
          T2[i][j][k][l] = s;
        }
  for (int I = 0; I < 6; ++I)
    for (int J = 0; J < 6; ++J) {
      static const int pi[6] = {0, 1, 2, 1, 0, 0}, pj[6] = {0, 1, 2, 2, 2, 1};
      out[6 * I + J] = T2[pi[I]][pj[I]][pi[J]][pj[J]];
    }
}

}  // namespace

// Used by the runtime to turn a crystal-frame material into grain frames.
void pf_rotate_voigt(const double* Cv, const double* R9, double* out) {
  double R[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) R[i][j] = R9[3 * i + j];
  rotate_voigt(Cv, R, out);
}

namespace {
// Unit plane normal m and shear direction s of variant vid (crystal frame,
// a = 1): m from the plane indices on the reciprocal basis, s from the
// direction indices on the direct one.
void variant_axes(double c_over_a, int vid, V3& m, V3& s) {
  const V3 a1{{std::sqrt(3.0) / 2.0, -0.5, 0.0}}, a2{{0.0, 1.0, 0.0}}, cc{{0.0, 0.0, c_over_a}};
  const V3 a3{{-(a1.v[0] + a2.v[0]), -(a1.v[1] + a2.v[1]), 0.0}};
  const double vol = dot(a1, cross(a2, cc));
  V3 b1 = cross(a2, cc), b2 = cross(cc, a1), b3 = cross(a1, a2);
  for (int k = 0; k < 3; ++k) {
    b1.v[k] /= vol;
    b2.v[k] /= vol;
    b3.v[k] /= vol;
  }
  const int* pl = kVariants[vid][0];
  const int* dr = kVariants[vid][1];
  m = unit(axpy(pl[0], b1, axpy(pl[1], b2, axpy(pl[3], b3, V3{{0, 0, 0}}))));
  s = unit(axpy(dr[0], a1, axpy(dr[1], a2, axpy(dr[2], a3, axpy(dr[3], cc, V3{{0, 0, 0}})))));
}
}  // namespace

extern "C" int pf_mg_twin_tables(const double C_hex[5], double c_over_a, double gamma_tw, int32_t n_grains,
                                 const double* rotations, int32_t n_var, const int32_t* variant_ids,
                                 double* C_grain, double* C_var, double* eps0) {
  if (!C_hex || !rotations || !variant_ids || !C_grain || !C_var || !eps0) return PF_EINVAL;
  if (n_grains < 1 || n_var < 1 || n_var > 6 || !(c_over_a > 0)) return PF_EINVAL;
  for (int q = 0; q < n_var; ++q)
    if (variant_ids[q] < 0 || variant_ids[q] > 5) return PF_EINVAL;
  const double C11 = C_hex[0], C12 = C_hex[1], C13 = C_hex[2], C33 = C_hex[3], C44 = C_hex[4];
  double Ch[36];
  std::memset(Ch, 0, sizeof(Ch));
  Ch[0] = Ch[7] = C11;
  Ch[14] = C33;
  Ch[1] = Ch[6] = C12;
  Ch[2] = Ch[12] = Ch[8] = Ch[13] = C13;
  Ch[21] = Ch[28] = C44;
  Ch[35] = 0.5 * (C11 - C12);
  for (int g = 0; g < n_grains; ++g) {
    double R[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) R[i][j] = rotations[9 * g + 3 * i + j];
    rotate_voigt(Ch, R, C_grain + 36 * g);
    for (int q = 0; q < n_var; ++q) {
      V3 m, s;
      variant_axes(c_over_a, variant_ids[q], m, s);
      double Q[3][3], Ctw[36];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Q[i][j] = 2.0 * m.v[i] * m.v[j] - (i == j ? 1.0 : 0.0);
      rotate_voigt(Ch, Q, Ctw);
      rotate_voigt(Ctw, R, C_var + 36 * ((size_t)g * n_var + q));
      // eps0 = gamma sym(s (x) m), rotated: R e R^T
      double e[3][3], er[3][3];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) e[i][j] = 0.5 * gamma_tw * (s.v[i] * m.v[j] + m.v[i] * s.v[j]);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          double acc = 0;
          for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l) acc += R[i][k] * R[j][l] * e[k][l];
          er[i][j] = acc;
        }
      double* o = eps0 + 6 * ((size_t)g * n_var + q);
      o[0] = er[0][0]; o[1] = er[1][1]; o[2] = er[2][2];
      o[3] = er[1][2]; o[4] = er[0][2]; o[5] = er[0][1];
    }
  }
  return PF_OK;
}

extern "C" int pf_mg_twin_gradient(double c_over_a, double c2n, double c2s, double c2t, int32_t n_grains,
                                   const double* rotations, int32_t n_var, const int32_t* variant_ids,
                                   double* kappa_var) {
  if (!rotations || !variant_ids || !kappa_var) return PF_EINVAL;
  if (n_grains < 1 || n_var < 1 || n_var > 6 || !(c_over_a > 0)) return PF_EINVAL;
  if (!(c2n >= 0) || !(c2s >= 0) || !(c2t >= 0)) return PF_EINVAL;
  for (int q = 0; q < n_var; ++q)
    if (variant_ids[q] < 0 || variant_ids[q] > 5) return PF_EINVAL;
  for (int g = 0; g < n_grains; ++g) {
    const double* R = rotations + 9 * g;
    for (int q = 0; q < n_var; ++q) {
      V3 m, s;
      variant_axes(c_over_a, variant_ids[q], m, s);
      const V3 t = cross(m, s);
      // sample-frame axes R m, R s, R t
      V3 ms{}, ss{}, ts{};
      for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) {
          ms.v[i] += R[3 * i + k] * m.v[k];
          ss.v[i] += R[3 * i + k] * s.v[k];
          ts.v[i] += R[3 * i + k] * t.v[k];
        }
      double K[3][3];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          K[i][j] = c2n * ms.v[i] * ms.v[j] + c2s * ss.v[i] * ss.v[j] + c2t * ts.v[i] * ts.v[j];
      double* o = kappa_var + 6 * ((size_t)g * n_var + q);
      o[0] = K[0][0]; o[1] = K[1][1]; o[2] = K[2][2];
      o[3] = K[1][2]; o[4] = K[0][2]; o[5] = K[0][1];
    }
  }
  return PF_OK;
}
