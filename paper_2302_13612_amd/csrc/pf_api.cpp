// Host runtime and C ABI of the phase-field twin step (see include/pf.h).
//
// A context holds one or more independent instances. Instances of one grid
// size form a group: their fields are stacked along z so that every pass
// over the group is one kernel launch, whatever the number of instances.
// A step of a group runs either
//   - the fixed-point path: Moulinec-Suquet iterations, then the driving
//     forces and the semi-implicit Allen-Cahn update; or
//   - the homogeneous spectral path, when an instance has one stiffness
//     everywhere, linear interpolation and no plastic strain: the
//     equilibrium is then known per wavevector and the step is one
//     forward and one inverse transform.
// When no group needs a host decision inside the step (no iterated fixed
// point, no profiling, no stress output), the launches of one step are
// captured once in a HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <functional>
#include <initializer_list>
#include <map>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/pf.h"
#include "pf_device.hpp"
#include "pf_fno.hpp"

void pf_rotate_voigt(const double* Cv, const double* R9, double* out);  // pf_crystal.cpp

using pft::DevState;
using pft::KArgs;
using pft::Status;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

// Workspace layout of one group (byte offsets from the group's base).
struct Layout {
  size_t eta, eps, eps_prev, eps_prev2, eps_prev3, sig, epsp, spec, tables, rot, ref, bss, loads, kh, khd, gk, tw;
  size_t part_rem, krem;
  size_t lapf;  // gradient force of the state (with a mobility field), else 0
  size_t pf_base, part_pc;  // fixed point over the update (pf_max_iter > 1), else 0
  size_t spec_bytes;        // size of the spectral buffer
  size_t part_ms, part_res, part_ac, part_mm, part_gd, state, total;
  int tab_stride;
};

int tab_stride_for(int nv) { return 21 * (nv + 1) + 6 * nv; }

bool axis_ok(int n) { return pfl::supported_axis(n); }

// A spectral component holds the rows of coefficients kx < nx/2, padded to a
// multiple of 16 complex values (128 bytes) so every 16-column tile of the y
// and z passes is one aligned cache line per row, then the Nyquist plane
// (kx = nx/2) as [inst][z][y]: keeping that one column in the rows would add a
// 16-wide tile of one useful column to every pass.
int spec_stride(int nx) { return (nx / 2 + 15) / 16 * 16; }

// Largest eigenvalue of a symmetric 3x3 matrix (tensor-Voigt xx yy zz yz xz
// xy) by the trigonometric closed form (O. K. Smith, Eigenvalues of a
// symmetric 3 x 3 matrix, Comm. ACM 4 (1961) 168).
double sym3_max_eigenvalue(const double* K) {
  const double a = K[0], b = K[1], c = K[2], d = K[3], e = K[4], f = K[5];
  const double p1 = d * d + e * e + f * f;
  if (p1 == 0.0) return std::max(a, std::max(b, c));
  const double q = (a + b + c) / 3.0;
  const double p2 = (a - q) * (a - q) + (b - q) * (b - q) + (c - q) * (c - q) + 2.0 * p1;
  const double p = std::sqrt(p2 / 6.0);
  // B = (K - q I) / p; r = det(B) / 2
  const double ba = (a - q) / p, bb = (b - q) / p, bc = (c - q) / p, bd = d / p, be = e / p, bf = f / p;
  const double det = ba * (bb * bc - bd * bd) - bf * (bf * bc - bd * be) + be * (bf * bd - bb * be);
  const double r = std::min(1.0, std::max(-1.0, 0.5 * det));
  return q + 2.0 * p * std::cos(std::acos(r) / 3.0);
}

// Spectral elements (complex) of one component of ninst instances.
size_t spec_comp(int nx, int ny, int nz, int ninst) {
  return (size_t)ny * nz * ninst * (spec_stride(nx) + 1);
}

void set_spec_layout(KArgs& a) {
  const size_t rows = (size_t)a.ny * a.nz * a.ninst;
  a.sh = spec_stride(a.nx);
  a.ncol = a.nx / 2;
  a.nq_row = 0;
  a.nqo = rows * a.sh;
  a.cs = spec_comp(a.nx, a.ny, a.nz, a.ninst);
}

// ninst instances of one size; own_epsp: the group keeps its own stacked
// plastic strain (batches), else the caller's buffer is used in place.
// mobile: a mobility field is given (the state's gradient force is kept and
// the spectra hold 2 nv components). picard: a fixed point over the update
// (the step's fixed base of the right-hand side and the per-block changes).
Layout make_layout(int nx, int ny, int nz, int nv, int n_grains, int ninst, bool own_epsp, bool mobile,
                   bool picard, bool grain_k) {
  Layout L{};
  const size_t nvox = (size_t)nx * ny * nz * ninst;
  const size_t nspec = spec_comp(nx, ny, nz, ninst);
  const int G = n_grains > 0 ? n_grains : 1;
  KArgs a{};
  a.nx = nx; a.ny = ny; a.nz = nz; a.nh = nx / 2 + 1; a.nv = nv; a.ninst = ninst;
  set_spec_layout(a);
  const size_t xb = (size_t)pfl::x_blocks(a);
  const size_t zb = (size_t)pfl::z_blocks(a, nv);
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
  L.eta = take(sizeof(float) * nvox * nv);
  L.eps = take(sizeof(float) * nvox * 6);
  L.eps_prev = take(sizeof(float) * nvox * 6);
  L.eps_prev2 = take(sizeof(float) * nvox * 6);
  L.eps_prev3 = take(sizeof(float) * nvox * 6);
  L.sig = take(sizeof(float) * nvox * 6);
  L.epsp = own_epsp ? take(sizeof(float) * nvox * 6) : 0;
  // six components (the fixed point's polarisation), 2V with a mobility
  // field, 3V for the macro-step residual of the spectral path (V <= 3)
  int ncomp = 6;
  if (mobile && 2 * nv > ncomp) ncomp = 2 * nv;
  if (nv <= pft::kKhMaxVar && 3 * nv > ncomp) ncomp = 3 * nv;
  if (grain_k && 4 * nv > ncomp) ncomp = 4 * nv;  // the update's V and the remainder's 3V
  L.spec_bytes = sizeof(float) * 2 * nspec * ncomp;
  L.spec = take(L.spec_bytes);
  L.lapf = mobile ? take(sizeof(float) * nvox * nv) : 0;
  // per-grain gradient tensors: the remainder's energy partials, the tables
  L.part_rem = grain_k ? take(sizeof(double) * xb) : 0;
  L.krem = grain_k ? take(sizeof(float) * 6 * (size_t)G * nv) : 0;
  L.pf_base = picard ? take(sizeof(float) * nvox * nv) : 0;
  L.part_pc = picard ? take(sizeof(float) * xb * 2) : 0;
  L.tab_stride = tab_stride_for(nv);
  L.tables = take(sizeof(float) * (size_t)L.tab_stride * G * ninst);
  L.rot = take(sizeof(float) * 12 * (size_t)G);
  L.ref = take(sizeof(float) * pft::kRefStride * (size_t)ninst);
  L.bss = take(sizeof(double) * 36 * (size_t)ninst);
  L.loads = take(sizeof(double) * 12 * (size_t)ninst);
  L.kh = take(sizeof(float) * pft::kKhStride * (size_t)ninst);
  L.khd = take(sizeof(double) * pft::kKhdStride * (size_t)ninst);
  L.gk = take(sizeof(float) * pft::kGkStride * (size_t)ninst);
  L.tw = take(sizeof(float) * 2 * (size_t)(nx / 2 + nx + ny + nz));
  L.part_ms = take(sizeof(double) * xb * pft::kQms);
  L.part_res = take(sizeof(double) * xb * pft::kQres);
  L.part_ac = take(sizeof(double) * xb * pft::kQac);
  L.part_mm = take(sizeof(float) * xb * 2);
  L.part_gd = take(sizeof(double) * zb * pft::kQgd);
  L.state = take(sizeof(DevState) * (size_t)ninst);
  L.total = off;
  return L;
}

// Invert an n x n matrix (row-major, double) by Gauss-Jordan with pivoting.
bool invert(int n, const double* A, double* out) {
  std::vector<double> m(n * 2 * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < 2 * n; ++j) m[i * 2 * n + j] = j < n ? A[i * n + j] : (j - n == i ? 1.0 : 0.0);
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(m[r * 2 * n + c]) > std::fabs(m[piv * 2 * n + c])) piv = r;
    if (m[piv * 2 * n + c] == 0.0) return false;
    if (piv != c)
      for (int j = 0; j < 2 * n; ++j) std::swap(m[c * 2 * n + j], m[piv * 2 * n + j]);
    const double d = m[c * 2 * n + c];
    for (int j = 0; j < 2 * n; ++j) m[c * 2 * n + j] /= d;
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = m[r * 2 * n + c];
      if (f != 0.0)
        for (int j = 0; j < 2 * n; ++j) m[r * 2 * n + j] -= f * m[c * 2 * n + j];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) out[i * n + j] = m[i * 2 * n + n + j];
  return true;
}

void pack_sym(const double* C, float* out) {
  for (int i = 0; i < 6; ++i)
    for (int j = i; j < 6; ++j) out[pft::sym6(i, j)] = (float)(0.5 * (C[6 * i + j] + C[6 * j + i]));
}

// Tensor-Voigt form of a Voigt stiffness: sigma = M eps with eps in tensor
// shear (M = C diag(1,1,1,2,2,2)), symmetrised.
void tensor_voigt(const double* C, double* M) {
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) M[6 * i + j] = 0.5 * (C[6 * i + j] + C[6 * j + i]) * (j < 3 ? 1.0 : 2.0);
}

// Inverse of the stress-controlled block of M, embedded in a 6x6 matrix.
bool stress_block_inverse(const double* M, uint32_t mask, double* out) {
  int idx[6], ns = 0;
  for (int i = 0; i < 6; ++i)
    if ((mask >> i) & 1u) idx[ns++] = i;
  for (int i = 0; i < 36; ++i) out[i] = 0.0;
  if (ns == 0) return true;
  double sub[36], inv[36];
  for (int i = 0; i < ns; ++i)
    for (int j = 0; j < ns; ++j) sub[i * ns + j] = M[6 * idx[i] + idx[j]];
  if (!invert(ns, sub, inv)) return false;
  for (int i = 0; i < ns; ++i)
    for (int j = 0; j < ns; ++j) out[6 * idx[i] + idx[j]] = inv[i * ns + j];
  return true;
}

// W_N^n = exp(-2 pi i n / N), computed in double, rounded once.
void twiddles(int N, float* out) {
  for (int n = 0; n < N; ++n) {
    const double ang = -2.0 * M_PI * (double)n / (double)N;
    out[2 * n] = (float)std::cos(ang);
    out[2 * n + 1] = (float)std::sin(ang);
  }
}

// Host-side preparation of one instance: sample-frame tables and everything
// derived from them.
struct InstanceHost {
  std::vector<float> tab;   // [G][tab_stride]
  std::vector<float> rot;   // [G][12]
  float ref[pft::kRefStride];
  double bss[36];
  float kh[pft::kKhStride];
  double khd[pft::kKhdStride];
  float gk[pft::kGkStride]; // gradient-energy coefficients (see kGkStride)
  bool aniso;               // kappa_var or kappa_grain given (gk holds K_a or kbar_a I)
  bool grain_k;             // kappa_grain given: krem holds K_a^g - kbar_a I
  std::vector<float> krem;  // [G][nv][6]
  bool one_iteration;       // one stiffness everywhere, equal to the reference
  bool homogeneous;         // one stiffness everywhere (spectral path possible)
};

int prepare_instance(const pf_problem* p, InstanceHost& h, std::string& why) {
  const int nv = p->n_var, G = p->n_grains;
  const bool rotated = p->grain_rot != nullptr;
  std::vector<double> Cg_s((size_t)36 * G), Cv_s((size_t)36 * G * nv), e0_s((size_t)6 * G * nv);
  for (int g = 0; g < G; ++g) {
    if (rotated) {
      const double* R = p->grain_rot + 9 * g;
      pf_rotate_voigt(p->C_grain, R, &Cg_s[36 * g]);
      for (int q = 0; q < nv; ++q) {
        pf_rotate_voigt(p->C_var + 36 * q, R, &Cv_s[36 * ((size_t)g * nv + q)]);
        const double* e = p->eps0 + 6 * q;
        const double A[3][3] = {{e[0], e[5], e[4]}, {e[5], e[1], e[3]}, {e[4], e[3], e[2]}};
        double B[3][3];
        for (int i = 0; i < 3; ++i)
          for (int k = 0; k < 3; ++k) {
            double acc = 0.0;
            for (int m = 0; m < 3; ++m)
              for (int n = 0; n < 3; ++n) acc += R[3 * i + m] * A[m][n] * R[3 * k + n];
            B[i][k] = acc;
          }
        double* o = &e0_s[6 * ((size_t)g * nv + q)];
        o[0] = B[0][0]; o[1] = B[1][1]; o[2] = B[2][2]; o[3] = B[1][2]; o[4] = B[0][2]; o[5] = B[0][1];
      }
    } else {
      std::memcpy(&Cg_s[36 * g], p->C_grain + 36 * g, 36 * sizeof(double));
      std::memcpy(&Cv_s[36 * (size_t)g * nv], p->C_var + 36 * (size_t)g * nv, 36 * nv * sizeof(double));
      std::memcpy(&e0_s[6 * (size_t)g * nv], p->eps0 + 6 * (size_t)g * nv, 6 * nv * sizeof(double));
    }
  }
  const int ts = tab_stride_for(nv);
  h.tab.assign((size_t)ts * G, 0.f);
  for (int g = 0; g < G; ++g) {
    float* t = h.tab.data() + (size_t)g * ts;
    const double* Cg = &Cg_s[36 * g];
    pack_sym(Cg, t);
    for (int q = 0; q < nv; ++q) {
      const double* Cv = &Cv_s[36 * ((size_t)g * nv + q)];
      double d[36];
      for (int i = 0; i < 36; ++i) d[i] = Cv[i] - Cg[i];
      pack_sym(d, t + 21 * (q + 1));
      for (int k = 0; k < 6; ++k) t[21 * (nv + 1) + 6 * q + k] = (float)e0_s[6 * ((size_t)g * nv + q) + k];
    }
  }
  h.rot.assign((size_t)12 * G, 0.f);
  if (rotated)
    for (int g = 0; g < G; ++g)
      for (int k = 0; k < 9; ++k) h.rot[12 * g + k] = (float)p->grain_rot[9 * g + k];
  // gradient energy: D_ij = 2 L dt K_ij c_i c_j and G_ij = K_ij c_i c_j with
  // c_i = 2 pi / (n_i dx), K = kappa I unless kappa_var gives K_a
  {
    const double tp = 2.0 * M_PI / p->dx;
    const double c[3] = {tp / p->nx, tp / p->ny, tp / p->nz};
    const double f = 2.0 * p->L * p->dt;
    std::memset(h.gk, 0, sizeof(h.gk));
    h.aniso = p->kappa_var != nullptr || p->kappa_grain != nullptr;
    h.grain_k = p->kappa_grain != nullptr;
    double kbar[pft::kMaxVar] = {};
    if (h.grain_k) {
      // the split of per-grain tensors: kbar_a I implicit, the rest explicit
      h.krem.assign((size_t)G * nv * 6, 0.f);
      for (int q = 0; q < nv; ++q)
        for (int g = 0; g < G; ++g) kbar[q] = std::max(kbar[q], sym3_max_eigenvalue(p->kappa_grain + 6 * ((size_t)g * nv + q)));
      for (int g = 0; g < G; ++g)
        for (int q = 0; q < nv; ++q)
          for (int k = 0; k < 6; ++k)
            h.krem[6 * ((size_t)g * nv + q) + k] =
                (float)(p->kappa_grain[6 * ((size_t)g * nv + q) + k] - (k < 3 ? kbar[q] : 0.0));
    }
    for (int q = 0; q < nv; ++q) {
      double K[6] = {p->kappa, p->kappa, p->kappa, 0.0, 0.0, 0.0};
      if (h.grain_k)
        K[0] = K[1] = K[2] = kbar[q];
      else if (h.aniso)
        for (int k = 0; k < 6; ++k) K[k] = p->kappa_var[6 * q + k];
      const double g[6] = {K[0] * c[0] * c[0], K[1] * c[1] * c[1], K[2] * c[2] * c[2],
                           2.0 * K[3] * c[1] * c[2], 2.0 * K[4] * c[0] * c[2], 2.0 * K[5] * c[0] * c[1]};
      for (int k = 0; k < 6; ++k) {
        h.gk[12 * q + k] = (float)(f * g[k]);
        h.gk[12 * q + 6 + k] = (float)g[k];
      }
    }
  }
  // reference medium
  double C0[36];
  if (p->C_ref_auto) {
    for (int i = 0; i < 36; ++i) {
      double s = 0.0;
      for (int g = 0; g < G; ++g) {
        s += Cg_s[36 * g + i];
        for (int q = 0; q < nv; ++q) s += Cv_s[36 * ((size_t)g * nv + q) + i];
      }
      C0[i] = s / (double)(G * (nv + 1));
    }
  } else {
    std::memcpy(C0, p->C_ref, sizeof(C0));
  }
  bool homog = (G == 1);
  for (int i = 0; i < 36 && homog; ++i)
    for (int q = 0; q < nv && homog; ++q)
      if (Cv_s[36 * q + i] != Cg_s[i]) homog = false;
  bool one = homog;
  for (int i = 0; i < 36 && one; ++i)
    if (Cg_s[i] != C0[i]) one = false;
  h.homogeneous = homog && !p->kappa_grain;
  h.one_iteration = one;
  pack_sym(C0, h.ref);
  double M0[36], S0[36];
  tensor_voigt(C0, M0);
  if (!invert(6, M0, S0)) {
    why = "reference stiffness is singular";
    return PF_EINVAL;
  }
  for (int i = 0; i < 36; ++i) h.ref[21 + i] = (float)S0[i];
  if (!stress_block_inverse(M0, p->bc_stress_mask, h.bss)) {
    why = "stress-controlled block of the reference stiffness is singular";
    return PF_EINVAL;
  }
  // spectral-path tables (grain 0)
  std::memset(h.kh, 0, sizeof(h.kh));
  std::memset(h.khd, 0, sizeof(h.khd));
  if (homog && nv <= pft::kKhMaxVar) {
    double M[36];
    tensor_voigt(&Cg_s[0], M);
    pack_sym(&Cg_s[0], h.kh);
    double s0[pft::kMaxVar][6];
    for (int q = 0; q < nv; ++q) {
      const double* e = &e0_s[6 * q];
      for (int i = 0; i < 6; ++i) {
        double acc = 0.0;
        for (int j = 0; j < 6; ++j) acc += M[6 * i + j] * e[j];
        s0[q][i] = acc;
        h.kh[21 + 6 * q + i] = (float)acc;
      }
    }
    for (int q = 0; q < nv; ++q)
      for (int r = 0; r < nv; ++r) {
        double w = 0.0;
        for (int c = 0; c < 6; ++c) w += (c < 3 ? 1.0 : 2.0) * s0[q][c] * e0_s[6 * r + c];
        h.kh[21 + 6 * pft::kMaxVar + nv * q + r] = (float)w;
      }
    std::memcpy(h.khd, M, sizeof(M));
    if (!stress_block_inverse(M, p->bc_stress_mask, h.khd + 36)) {
      why = "stress-controlled block of the stiffness is singular";
      return PF_EINVAL;
    }
    for (int q = 0; q < nv; ++q)
      for (int c = 0; c < 6; ++c) h.khd[72 + 6 * q + c] = e0_s[6 * q + c];
  }
  return PF_OK;
}

struct ProfEntry {
  std::string name;
  hipEvent_t start, stop;
};

// One group of same-size instances.
struct Group {
  int nx, ny, nz, nh, ninst;
  size_t nvox;           // voxels per instance
  size_t base;           // workspace offset
  Layout L;
  KArgs args;
  bool one_iteration;    // every instance exact after one fixed-point iteration
  bool homogeneous;      // every instance eligible for the spectral path
  bool strain_valid;     // the strain field describes the current state
  int64_t hist;          // consecutive fixed-point steps with a valid strain history
  bool own_epsp, epsp_given;
  bool mobile;           // a mobility field (one instance): generic path only
  bool lap_valid;        // the kept gradient force matches the order parameters
  int pf_max_iter;       // solves of the update's fixed point per step (1: plain step)
  double pf_tol;         // its stopping threshold on max |f^i - f^{i-1}|
  std::vector<int> members;
  float* ring[4];        // strain fields: ring[cur] the latest converged one, then
  int cur;               // ring[cur - 1], ring[cur - 2], ring[cur - 3] those of the steps before
  int last_iters;        // fixed-point iterations of the group's last step (most of its instances')
  int32_t fin_seq;       // status publications enqueued for each instance (k_fin_res launches)
  size_t status_off;     // index of its first instance in the host status array
};

}  // namespace

struct pf_ctx {
  int nv, n_inst;
  double dx, kappa;
  hipStream_t stream;
  char* ws;
  std::vector<Group> groups;
  std::vector<std::pair<int, int>> where;  // instance -> (group, index in group)
  int ms_max_iter;
  uint32_t stress_mask;
  int h_kind;
  int64_t steps;
  int64_t steps_replayed;  // fixed-point steps replayed as one graph
  Status* host_status;   // pinned, [n_inst]
  double* host_loads;    // pinned, [n_inst][12]
  bool loads_uploaded;
  std::string err;
  // graph replay of one step
  hipStream_t cap_stream;
  hipGraphExec_t gexec;
  std::string gkey;
  // graphs of single steps whose fixed point runs on the device, by key
  std::map<std::string, hipGraphExec_t> sgraphs;
  bool capturing;
  // profiling
  bool prof_on;
  std::string prof_only;  // time only the launches of this stage ("" = all)
  std::vector<ProfEntry> prof;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::string> prof_names;
  std::vector<int64_t> prof_counts;
  std::vector<double> prof_ms;
};

namespace {

int fail(pf_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

int hip_fail(pf_ctx* c, hipError_t e, const char* what) {
  return fail(c, PF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

hipEvent_t get_event(pf_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  // timing-only events: no system-scope fence when they are recorded (the
  // fence writes back the caches and stretches the timed launch)
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

// Launch one stage on stream s, bracketed by events when profiling is on.
template <class F>
int launch(pf_ctx* c, hipStream_t s, const char* name, F&& f) {
  ProfEntry pe;
  const bool prof = c->prof_on && !c->capturing && (c->prof_only.empty() || c->prof_only == name);
  if (prof) {
    pe.name = name;
    pe.start = get_event(c);
    pe.stop = get_event(c);
    if (pe.start) hipEventRecord(pe.start, s);
  }
  hipError_t e = f();
  if (e != hipSuccess) return hip_fail(c, e, name);
  if (prof && pe.start && pe.stop) {
    hipEventRecord(pe.stop, s);
    c->prof.push_back(pe);
  }
  return PF_OK;
}

#define PF_TRY(expr)          \
  do {                        \
    int _rc = (expr);         \
    if (_rc != PF_OK) return _rc; \
  } while (0)

int validate(const pf_problem* p, std::string& why) {
  if (!p) { why = "null problem"; return PF_EINVAL; }
  if (!axis_ok(p->nx) || !axis_ok(p->ny) || !axis_ok(p->nz)) {
    why = "grid sizes must each be one of 32, 48, 64, 96, 128, 192, 256, 384, 512";
    return PF_EINVAL;
  }
  if (p->n_var < 1 || p->n_var > pft::kMaxVar) { why = "n_var must be in 1..6"; return PF_EINVAL; }
  if (p->n_grains < 1 || p->n_grains > 255) { why = "n_grains must be in 1..255"; return PF_EINVAL; }
  if (p->n_grains > 1 && !p->grain_id) { why = "grain_id required when n_grains > 1"; return PF_EINVAL; }
  if (!p->C_grain || !p->C_var || !p->eps0) { why = "material tables required"; return PF_EINVAL; }
  if (!p->eta0) { why = "eta0 required"; return PF_EINVAL; }
  if (!(p->dx > 0) || !(p->L >= 0) || !(p->dt > 0) || !(p->kappa >= 0) || !(p->A >= 0)) {
    why = "dx, dt must be > 0 and A, kappa, L >= 0";
    return PF_EINVAL;
  }
  if (p->h_kind != PF_H_LINEAR && p->h_kind != PF_H_QUINTIC) { why = "bad h_kind"; return PF_EINVAL; }
  if (p->ms_max_iter < 1) { why = "ms_max_iter must be >= 1"; return PF_EINVAL; }
  if (!(p->ms_tol >= 0)) { why = "ms_tol must be >= 0"; return PF_EINVAL; }
  if (p->pf_max_iter < 0) { why = "pf_max_iter must be >= 0"; return PF_EINVAL; }
  if (p->pf_max_iter > 1 && !(p->pf_tol >= 0 && std::isfinite(p->pf_tol))) {
    why = "pf_tol must be finite and >= 0";
    return PF_EINVAL;
  }
  if (p->bc_stress_mask > 63u) { why = "bc_stress_mask has bits above 5"; return PF_EINVAL; }
  if (p->kappa_var) {
    for (int q = 0; q < p->n_var; ++q) {
      const double* K = p->kappa_var + 6 * q;
      for (int k = 0; k < 6; ++k)
        if (!std::isfinite(K[k])) { why = "kappa_var must be finite"; return PF_EINVAL; }
      if (K[0] < 0 || K[1] < 0 || K[2] < 0) { why = "kappa_var diagonal must be >= 0"; return PF_EINVAL; }
    }
    if (p->n_grains != 1) {
      why = "an anisotropic gradient energy (kappa_var) needs one grain; kappa_grain takes one tensor per grain";
      return PF_EUNSUPPORTED;
    }
  }
  if (p->kappa_grain) {
    if (p->kappa_var) { why = "kappa_var and kappa_grain exclude each other"; return PF_EINVAL; }
    for (size_t i = 0; i < (size_t)p->n_grains * p->n_var; ++i) {
      const double* K = p->kappa_grain + 6 * i;
      for (int k = 0; k < 6; ++k)
        if (!std::isfinite(K[k])) { why = "kappa_grain must be finite"; return PF_EINVAL; }
      if (K[0] < 0 || K[1] < 0 || K[2] < 0) { why = "kappa_grain diagonal must be >= 0"; return PF_EINVAL; }
    }
    if (p->mobility) { why = "kappa_grain does not combine with a mobility field"; return PF_EUNSUPPORTED; }
    if (p->pf_max_iter > 1) {
      why = "kappa_grain does not combine with the fixed point over the update (pf_max_iter > 1)";
      return PF_EUNSUPPORTED;
    }
  }
  return PF_OK;
}

// Batch-wide checks: what the instances of one context must share.
int validate_batch(const pf_problem* probs, int n, std::string& why) {
  if (!probs || n < 1) { why = "need at least one problem"; return PF_EINVAL; }
  for (int i = 0; i < n; ++i) {
    const int rc = validate(&probs[i], why);
    if (rc != PF_OK) {
      why = "instance " + std::to_string(i) + ": " + why;
      return rc;
    }
  }
  // the x passes address a field component with 32-bit element offsets
  for (int i = 0; i < n; ++i) {
    size_t same = 0;
    for (int j = 0; j < n; ++j)
      if (probs[j].nx == probs[i].nx && probs[j].ny == probs[i].ny && probs[j].nz == probs[i].nz) ++same;
    if (same * (size_t)probs[i].nx * probs[i].ny * probs[i].nz >= ((size_t)1 << 30)) {
      why = "instances of one grid size must hold fewer than 2^30 voxels together";
      return PF_EINVAL;
    }
  }
  if (n == 1) return PF_OK;
  for (int i = 0; i < n; ++i) {
    if (probs[i].mobility) {
      why = "a mobility field needs a one-instance context";
      return PF_EUNSUPPORTED;
    }
    if (probs[i].kappa_grain) {
      why = "per-grain gradient tensors (kappa_grain) need a one-instance context";
      return PF_EUNSUPPORTED;
    }
    if (probs[i].pf_max_iter > 1) {
      why = "a fixed point over the update (pf_max_iter > 1) needs a one-instance context";
      return PF_EUNSUPPORTED;
    }
  }
  const pf_problem& p0 = probs[0];
  for (int i = 0; i < n; ++i) {
    const pf_problem& p = probs[i];
    if (p.n_grains != 1) { why = "batched instances must each be one grain"; return PF_EINVAL; }
    if (p.n_var != p0.n_var || p.h_kind != p0.h_kind || p.A != p0.A || p.kappa != p0.kappa || p.L != p0.L ||
        p.dt != p0.dt || p.dx != p0.dx || p.ms_tol != p0.ms_tol || p.ms_max_iter != p0.ms_max_iter ||
        p.bc_stress_mask != p0.bc_stress_mask) {
      why = "batched instances must share n_var, h_kind, A, kappa, L, dt, dx, ms_tol, ms_max_iter and "
            "bc_stress_mask";
      return PF_EINVAL;
    }
  }
  return PF_OK;
}

// Group the instances by grid size, in order of first appearance.
std::vector<Group> plan_groups(const pf_problem* probs, int n) {
  std::vector<Group> gs;
  for (int i = 0; i < n; ++i) {
    const pf_problem& p = probs[i];
    size_t k = 0;
    while (k < gs.size() && !(gs[k].nx == p.nx && gs[k].ny == p.ny && gs[k].nz == p.nz)) ++k;
    if (k == gs.size()) {
      Group g{};
      g.nx = p.nx; g.ny = p.ny; g.nz = p.nz; g.nh = p.nx / 2 + 1;
      g.nvox = (size_t)p.nx * p.ny * p.nz;
      gs.push_back(g);
    }
    gs[k].members.push_back(i);
  }
  size_t off = 0;
  for (auto& g : gs) {
    g.ninst = (int)g.members.size();
    g.own_epsp = n > 1;
    g.mobile = probs[g.members[0]].mobility != nullptr;
    g.pf_max_iter = std::max(1, (int)probs[g.members[0]].pf_max_iter);
    g.pf_tol = probs[g.members[0]].pf_tol;
    g.L = make_layout(g.nx, g.ny, g.nz, probs[0].n_var, probs[g.members[0]].n_grains, g.ninst, g.own_epsp,
                      g.mobile, g.pf_max_iter > 1, probs[g.members[0]].kappa_grain != nullptr);
    g.base = off;
    off += g.L.total;
  }
  return gs;
}

size_t batch_bytes(const pf_problem* probs, int n) {
  size_t total = 0;
  for (auto& g : plan_groups(probs, n)) total += g.L.total;
  return total;
}

int read_status(pf_ctx* c) {
  size_t off = 0;
  for (auto& g : c->groups) {
    hipError_t e = hipMemcpy2DAsync(c->host_status + off, sizeof(Status), &g.args.state->st, sizeof(DevState),
                                    sizeof(Status), g.ninst, hipMemcpyDeviceToHost, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "status copy");
    off += g.ninst;
  }
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "stream sync");
  return PF_OK;
}

// Wait until the fixed point's finalize of every instance of the given
// groups has published its status (seq reached the launches enqueued), by
// polling the host-visible array; a stream that went idle without it (or an
// error) falls back to copying the status.
int wait_published(pf_ctx* c, const std::vector<size_t>& groups) {
  for (int spin = 0;; ++spin) {
    bool all = true;
    for (size_t k : groups) {
      const Group& g = c->groups[k];
      for (int j = 0; j < g.ninst && all; ++j) {
        const int seq = __atomic_load_n(&c->host_status[g.status_off + j].seq, __ATOMIC_ACQUIRE);
        all = seq == g.fin_seq;
      }
      if (!all) break;
    }
    if (all) return PF_OK;
    if ((spin & 1023) == 1023) {
      const hipError_t q = hipStreamQuery(c->stream);
      if (q == hipSuccess) return read_status(c);
      if (q != hipErrorNotReady) return hip_fail(c, q, "stream query");
    }
  }
}

// host_status index range of a group
size_t status_base(pf_ctx* c, size_t gi) {
  size_t off = 0;
  for (size_t k = 0; k < gi; ++k) off += c->groups[k].ninst;
  return off;
}

int ms_iteration(pf_ctx* c, const KArgs& a, hipStream_t s) {
  PF_TRY(launch(c, s, "ms_x_forward", [&] { return pfl::ms_x_forward(a, s); }));
  PF_TRY(launch(c, s, "ms_y_forward", [&] { return pfl::y_pass(a, 6, 1, s); }));
  PF_TRY(launch(c, s, "ms_z_green", [&] { return pfl::ms_z_green(a, s); }));
  PF_TRY(launch(c, s, "ms_y_inverse", [&] { return pfl::y_pass(a, 6, -1, s); }));
  PF_TRY(launch(c, s, "ms_x_inverse", [&] { return pfl::ms_x_inverse(a, s); }));
  PF_TRY(launch(c, s, "ms_finalize_residual", [&] { return pfl::ms_finalize_residual(a, s); }));
  return PF_OK;
}

// The update of a step. With pf_max_iter > 1 it is the fixed point i of
// Table 1 (eqs. (19)-(20)): the guess is f^n, every further solve takes the
// chemical force of the latest iterate (pc_x_forward) while the gradient
// term stays implicit and the mechanical force stays that of f^n; after each
// solve the host reads max |f^i - f^{i-1}| and stops at pf_tol.
// Per-grain gradient tensors, first part of the explicit remainder
// 2 div((K(x) - kbar I) grad f^n): the gradient of the order parameters and
// the flux (K - kbar I) grad f (with its energy into a.part_rem), held after
// their x and y transforms in the spectral components V .. 4V-1; the update's
// divergence pass (k_z_div) adds the rest after the update's y transform.
int remainder_flux(pf_ctx* c, const KArgs& a, hipStream_t s) {
  const int V = a.nv;
  KArgs r = a;
  r.spec = a.spec + (size_t)V * a.cs;  // components V .. 4V-1
  PF_TRY(launch(c, s, "rem_x_forward", [&] { return pfl::raw_x_forward(r, a.eta, V, s); }));
  PF_TRY(launch(c, s, "rem_y_forward", [&] { return pfl::y_pass(r, V, 1, s); }));
  PF_TRY(launch(c, s, "rem_z_gradient", [&] { return pfl::grad_z(r, s); }));
  PF_TRY(launch(c, s, "rem_y_inverse3", [&] { return pfl::y_pass(r, 3 * V, -1, s); }));
  PF_TRY(launch(c, s, "rem_x_flux", [&] { return pfl::flux_x(r, s); }));
  PF_TRY(launch(c, s, "rem_y_forward3", [&] { return pfl::y_pass(r, 3 * V, 1, s); }));
  return PF_OK;
}

int ac_update_args(pf_ctx* c, const Group& g, const KArgs& a, hipStream_t s) {
  if (a.krem) PF_TRY(remainder_flux(c, a, s));
  PF_TRY(launch(c, s, "ac_x_forward", [&] { return pfl::ac_x_forward(a, s); }));
  for (int it = 1;; ++it) {
    PF_TRY(launch(c, s, "ac_y_forward", [&] { return pfl::y_pass(a, a.nv, 1, s); }));
    if (a.krem) PF_TRY(launch(c, s, "rem_z_divergence", [&] { return pfl::div_z(a, s); }));
    PF_TRY(launch(c, s, "ac_z_update", [&] { return pfl::ac_z_update(a, 0, s); }));
    PF_TRY(launch(c, s, "ac_y_inverse", [&] { return pfl::y_pass(a, a.lapf ? 2 * a.nv : a.nv, -1, s); }));
    PF_TRY(launch(c, s, "ac_x_inverse", [&] { return pfl::ac_x_inverse(a, s); }));
    if (g.pf_max_iter <= 1) break;
    PF_TRY(launch(c, s, "pc_finalize", [&] { return pfl::pc_finalize(a, it, s); }));
    PF_TRY(read_status(c));
    const size_t b = status_base(c, (size_t)(&g - c->groups.data()));
    const double change = c->host_status[b].pf_change;
    if (change <= g.pf_tol) break;
    if (it == g.pf_max_iter) {
      char buf[160];
      snprintf(buf, sizeof(buf), "phase-field fixed point not converged after %d solves (change %.3e)", it,
               change);
      return fail(c, PF_ENOCONV, buf);
    }
    PF_TRY(launch(c, s, "pc_x_forward", [&] { return pfl::pc_x_forward(a, s); }));
  }
  PF_TRY(launch(c, s, "ac_finalize", [&] { return pfl::ac_finalize(a, 0, s); }));
  return PF_OK;
}

int ac_update(pf_ctx* c, const Group& g, hipStream_t s) { return ac_update_args(c, g, g.args, s); }

// The statistics of the homogeneous spectral path (reductions of the step's
// passes); needed after the last step of a call only: every pass of a step
// reduces what that step needs itself.
int kh_finalize(pf_ctx* c, const Group& g, hipStream_t s) {
  const KArgs& a = g.args;
  return launch(c, s, "kh_finalize", [&] { return pfl::ac_finalize(a, 2, s); });
}

// The whole homogeneous spectral step of a group (statistics on request).
int kh_step(pf_ctx* c, const Group& g, bool fin, hipStream_t s) {
  const KArgs& a = g.args;
  PF_TRY(launch(c, s, "kh_x_forward", [&] { return pfl::kh_x_forward(a, 0, s); }));
  PF_TRY(launch(c, s, "kh_y_forward", [&] { return pfl::y_pass(a, 2 * a.nv, 1, s); }));
  PF_TRY(launch(c, s, "kh_z_update", [&] { return pfl::kh_z_update(a, 0, s); }));
  PF_TRY(launch(c, s, "kh_y_inverse", [&] { return pfl::y_pass(a, a.nv, -1, s); }));
  PF_TRY(launch(c, s, "kh_x_inverse", [&] { return pfl::ac_x_inverse(a, s); }));
  if (fin) PF_TRY(kh_finalize(c, g, s));
  return PF_OK;
}

// One step of a group that needs no host decision (spectral path or one
// fixed-point iteration); fin: the spectral path's statistics too.
int fixed_step(pf_ctx* c, const Group& g, bool kh, bool fin, hipStream_t s) {
  if (kh) return kh_step(c, g, fin, s);
  KArgs ab = g.args;
  ab.iter_mode = 0;
  PF_TRY(launch(c, s, "step_begin", [&] { return pfl::step_begin(ab, s); }));
  PF_TRY(ms_iteration(c, ab, s));
  return ac_update(c, g, s);
}

void drop_graph(pf_ctx* c) {
  if (c->gexec) hipGraphExecDestroy(c->gexec);
  c->gexec = nullptr;
  c->gkey.clear();
  for (auto& kv : c->sgraphs) hipGraphExecDestroy(kv.second);
  c->sgraphs.clear();
}

// Replay the graph of one step under key, capturing it with build(stream)
// first if it is not cached (at most kMaxStepGraphs are kept).
constexpr size_t kMaxStepGraphs = 32;
template <class F>
int run_step_graph(pf_ctx* c, const std::string& key, F&& build) {
  hipError_t e;
  auto it = c->sgraphs.find(key);
  if (it == c->sgraphs.end()) {
    if (c->sgraphs.size() >= kMaxStepGraphs) {
      for (auto& kv : c->sgraphs) hipGraphExecDestroy(kv.second);
      c->sgraphs.clear();
    }
    if (!c->cap_stream) {
      if ((e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(c, e, "capture stream");
    }
    if ((e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed)) != hipSuccess)
      return hip_fail(c, e, "begin capture");
    c->capturing = true;
    const int rc = build(c->cap_stream);
    c->capturing = false;
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(c->cap_stream, &graph);
    if (rc != PF_OK) {
      if (graph) hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(c, e, "end capture");
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(c, e, "graph instantiate");
    it = c->sgraphs.emplace(key, ex).first;
  }
  if ((e = hipGraphLaunch(it->second, c->stream)) != hipSuccess) return hip_fail(c, e, "graph launch");
  return PF_OK;
}

// Capture (or reuse) the graph of one step of every group and replay it.
int run_graph(pf_ctx* c, int n_steps, const std::vector<char>& use_kh, const std::string& key) {
  hipError_t e;
  if (!c->gexec || c->gkey != key) {
    drop_graph(c);
    if (!c->cap_stream) {
      if ((e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(c, e, "capture stream");
    }
    if ((e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed)) != hipSuccess)
      return hip_fail(c, e, "begin capture");
    c->capturing = true;
    int rc = PF_OK;
    for (size_t k = 0; k < c->groups.size() && rc == PF_OK; ++k)
      rc = fixed_step(c, c->groups[k], use_kh[k] != 0, false, c->cap_stream);
    c->capturing = false;
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(c->cap_stream, &graph);
    if (rc != PF_OK) {
      if (graph) hipGraphDestroy(graph);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(c, e, "end capture");
    e = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e != hipSuccess) {
      c->gexec = nullptr;
      return hip_fail(c, e, "graph instantiate");
    }
    c->gkey = key;
  }
  for (int n = 0; n < n_steps; ++n)
    if ((e = hipGraphLaunch(c->gexec, c->stream)) != hipSuccess) return hip_fail(c, e, "graph launch");
  for (size_t k = 0; k < c->groups.size(); ++k)
    if (use_kh[k]) PF_TRY(kh_finalize(c, c->groups[k], c->stream));
  return PF_OK;
}

// Loads -> device through the pinned staging buffer (free at the start of a
// call: every call that used it ended with a synchronisation of the stream).
int upload_loads(pf_ctx* c, const pf_load* loads) {
  hipError_t e;
  bool changed = !c->loads_uploaded;
  for (int i = 0; i < c->n_inst; ++i) {
    double* h = c->host_loads + 12 * (size_t)i;
    for (int k = 0; k < 6; ++k) {
      if (h[k] != loads[i].eps_bar[k] || h[6 + k] != loads[i].sig_bar[k]) changed = true;
    }
  }
  if (changed) {
    e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "stream sync");
    for (auto& g : c->groups) {
      for (size_t j = 0; j < g.members.size(); ++j) {
        double* h = c->host_loads + 12 * (size_t)g.members[j];
        const pf_load& ld = loads[g.members[j]];
        for (int k = 0; k < 6; ++k) {
          h[k] = ld.eps_bar[k];
          h[6 + k] = ld.sig_bar[k];
        }
      }
    }
    for (auto& g : c->groups)
      for (size_t j = 0; j < g.members.size(); ++j) {
        e = hipMemcpyAsync(const_cast<double*>(g.args.loads) + 12 * j, c->host_loads + 12 * (size_t)g.members[j],
                           sizeof(double) * 12, hipMemcpyHostToDevice, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "load copy");
      }
    c->loads_uploaded = true;
  }
  return PF_OK;
}

// Gradient energy of the group's current order parameters (reported by the
// next step's stats) after they were replaced from outside a step.
int refresh_gradient_energy(pf_ctx* c, const Group& g) {
  const KArgs& a = g.args;
  hipStream_t s = c->stream;
  PF_TRY(launch(c, s, "init_x", [&] { return pfl::raw_x_forward(a, a.eta, c->nv, s); }));
  PF_TRY(launch(c, s, "init_y", [&] { return pfl::y_pass(a, c->nv, 1, s); }));
  PF_TRY(launch(c, s, "init_z", [&] { return pfl::ac_z_update(a, 1, s); }));
  PF_TRY(launch(c, s, "init_fin", [&] { return pfl::ac_finalize(a, 1, s); }));
  return PF_OK;
}

// The gradient force 2 div(K grad f) of the current order parameters, which
// a step with a mobility field reads (each such step leaves that of its new
// state); needed after init and after the order parameters were replaced.
int refresh_gradient_force(pf_ctx* c, const Group& g) {
  const KArgs& a = g.args;
  hipStream_t s = c->stream;
  PF_TRY(launch(c, s, "lap_x", [&] { return pfl::raw_x_forward(a, a.eta, c->nv, s); }));
  PF_TRY(launch(c, s, "lap_y", [&] { return pfl::y_pass(a, c->nv, 1, s); }));
  PF_TRY(launch(c, s, "lap_z", [&] { return pfl::ac_z_update(a, 2, s); }));
  PF_TRY(launch(c, s, "lap_y_inverse", [&] { return pfl::y_pass(a, c->nv, -1, s); }));
  PF_TRY(launch(c, s, "lap_x_inverse", [&] { return pfl::raw_x_inverse(a, a.lapf, c->nv, 1.f, s); }));
  return PF_OK;
}

int check_instance(pf_ctx* c, int32_t inst) {
  if (inst < 0 || inst >= c->n_inst) return fail(c, PF_EINVAL, "instance index out of range");
  return PF_OK;
}

}  // namespace

extern "C" {

int pf_batch_workspace_size(const pf_problem* probs, int32_t n_inst, size_t* bytes) {
  if (!bytes) return PF_EINVAL;
  std::string why;
  if (validate_batch(probs, n_inst, why) != PF_OK) return PF_EINVAL;
  *bytes = batch_bytes(probs, n_inst);
  return PF_OK;
}

int pf_workspace_size(const pf_problem* p, size_t* bytes) {
  if (!bytes) return PF_EINVAL;
  if (!p || !axis_ok(p->nx) || !axis_ok(p->ny) || !axis_ok(p->nz) || p->n_var < 1 ||
      p->n_var > pft::kMaxVar || p->n_grains < 1 || p->n_grains > 255)
    return PF_EINVAL;
  *bytes = batch_bytes(p, 1);
  return PF_OK;
}

int pf_batch_init(const pf_problem* probs, int32_t n_inst, void* workspace, size_t ws_bytes, void* hip_stream,
                  pf_ctx** out) {
  if (!out) return PF_EINVAL;
  *out = nullptr;
  std::string why;
  int rc = validate_batch(probs, n_inst, why);
  if (rc != PF_OK) {
    fprintf(stderr, "pf_init: %s\n", why.c_str());
    return rc;
  }
  std::vector<Group> groups = plan_groups(probs, n_inst);
  size_t need = 0;
  for (auto& g : groups) need += g.L.total;
  if (!workspace || ws_bytes < need) {
    fprintf(stderr, "pf_init: workspace of %zu bytes needed\n", need);
    return PF_ENOMEM;
  }
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0) {
    fprintf(stderr, "pf_init: workspace must be 256-byte aligned\n");
    return PF_EINVAL;
  }
  std::vector<InstanceHost> hosts(n_inst);
  for (int i = 0; i < n_inst; ++i) {
    rc = prepare_instance(&probs[i], hosts[i], why);
    if (rc != PF_OK) {
      fprintf(stderr, "pf_init: instance %d: %s\n", i, why.c_str());
      return rc;
    }
  }
  pf_ctx* c = new (std::nothrow) pf_ctx();
  if (!c) return PF_ENOMEM;
  const pf_problem& p0 = probs[0];
  c->nv = p0.n_var;
  c->n_inst = n_inst;
  c->dx = p0.dx;
  c->kappa = p0.kappa;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  c->ws = static_cast<char*>(workspace);
  c->ms_max_iter = p0.ms_max_iter;
  c->stress_mask = p0.bc_stress_mask;
  c->h_kind = p0.h_kind;
  c->steps = 0;
  c->steps_replayed = 0;
  c->loads_uploaded = false;
  c->cap_stream = nullptr;
  c->gexec = nullptr;
  c->capturing = false;
  c->prof_on = false;
  c->groups = groups;
  c->where.resize(n_inst);
  for (size_t k = 0; k < c->groups.size(); ++k)
    for (size_t j = 0; j < c->groups[k].members.size(); ++j) c->where[c->groups[k].members[j]] = {(int)k, (int)j};

  hipError_t e;
  c->host_status = nullptr;
  c->host_loads = nullptr;
  auto bail = [&](hipError_t err, const char* what) {
    fprintf(stderr, "pf_init: %s: %s\n", what, hipGetErrorString(err));
    if (c->host_status) hipHostFree(c->host_status);
    if (c->host_loads) hipHostFree(c->host_loads);
    delete c;
    return PF_EDEVICE;
  };
  // the status array is written by the device directly (fine-grained, mapped)
  if ((e = hipHostMalloc(reinterpret_cast<void**>(&c->host_status), sizeof(Status) * n_inst,
                         hipHostMallocMapped | hipHostMallocCoherent)) != hipSuccess)
    return bail(e, "hipHostMalloc");
  Status* status_dev = nullptr;
  if ((e = hipHostGetDevicePointer(reinterpret_cast<void**>(&status_dev), c->host_status, 0)) != hipSuccess)
    return bail(e, "hipHostGetDevicePointer");
  if ((e = hipHostMalloc(reinterpret_cast<void**>(&c->host_loads), sizeof(double) * 12 * n_inst,
                         hipHostMallocDefault)) != hipSuccess)
    return bail(e, "hipHostMalloc");
  std::memset(c->host_status, 0, sizeof(Status) * n_inst);
  std::memset(c->host_loads, 0, sizeof(double) * 12 * n_inst);

  const int nv = p0.n_var;
  size_t status_off = 0;
  for (auto& g : c->groups) {
    const Layout& L = g.L;
    const pf_problem& pg = probs[g.members[0]];
    const int G = pg.n_grains;
    g.one_iteration = true;
    g.homogeneous = nv <= pft::kKhMaxVar && p0.h_kind == PF_H_LINEAR;
    for (int m : g.members) {
      g.one_iteration = g.one_iteration && hosts[m].one_iteration;
      g.homogeneous = g.homogeneous && hosts[m].homogeneous;
    }
    g.strain_valid = true;
    g.hist = 0;
    g.epsp_given = false;
    char* ws = c->ws + g.base;
    KArgs& a = g.args;
    std::memset(&a, 0, sizeof(a));
    a.nx = g.nx; a.ny = g.ny; a.nz = g.nz; a.nh = g.nh; a.nv = nv;
    a.ninst = g.ninst;
    set_spec_layout(a);
    a.h_kind = p0.h_kind;
    a.n_grains = G;
    a.tab_stride = L.tab_stride;
    a.tab_inst = L.tab_stride * G;
    a.A = (float)p0.A;
    a.LDt = (float)(p0.L * p0.dt);
    const double twopi = 2.0 * M_PI;
    const double kx = twopi / (g.nx * p0.dx), ky = twopi / (g.ny * p0.dx), kz = twopi / (g.nz * p0.dx);
    const double f = 2.0 * p0.L * p0.dt * p0.kappa;
    a.ax = (float)(f * kx * kx); a.ay = (float)(f * ky * ky); a.az = (float)(f * kz * kz);
    a.gx = kx * kx; a.gy = ky * ky; a.gz = kz * kz;
    a.cdx = (float)kx; a.cdy = (float)ky; a.cdz = (float)kz;
    a.inv_ntot = (float)(1.0 / (double)g.nvox);
    a.tol = p0.ms_tol;
    a.stress_mask = p0.bc_stress_mask;
    a.eta = reinterpret_cast<float*>(ws + L.eta);
    g.ring[0] = reinterpret_cast<float*>(ws + L.eps);
    g.ring[1] = reinterpret_cast<float*>(ws + L.eps_prev);
    g.ring[2] = reinterpret_cast<float*>(ws + L.eps_prev2);
    g.ring[3] = reinterpret_cast<float*>(ws + L.eps_prev3);
    g.cur = 0;
    g.last_iters = 0;
    g.fin_seq = 0;
    a.eps = a.eps_out = g.ring[0];
    a.eps_h1 = a.eps_h2 = a.eps_h3 = nullptr;
    a.iter_mode = 0;
    a.sig = reinterpret_cast<float*>(ws + L.sig);
    a.epsp = nullptr;
    a.gid = G > 1 ? pg.grain_id : nullptr;
    a.tables = reinterpret_cast<float*>(ws + L.tables);
    a.ref = reinterpret_cast<float*>(ws + L.ref);
    a.bss = reinterpret_cast<double*>(ws + L.bss);
    a.loads = reinterpret_cast<double*>(ws + L.loads);
    a.kh = reinterpret_cast<float*>(ws + L.kh);
    a.khd = reinterpret_cast<double*>(ws + L.khd);
    bool aniso = false;
    for (int m : g.members) aniso = aniso || hosts[m].aniso;
    a.gk = aniso ? reinterpret_cast<float*>(ws + L.gk) : nullptr;
    a.mob = g.mobile ? pg.mobility : nullptr;
    a.lapf = g.mobile ? reinterpret_cast<float*>(ws + L.lapf) : nullptr;
    const bool grain_k = hosts[g.members[0]].grain_k;
    a.part_rem = grain_k ? reinterpret_cast<double*>(ws + L.part_rem) : nullptr;
    a.krem = grain_k ? reinterpret_cast<const float*>(ws + L.krem) : nullptr;
    a.pf_base = g.pf_max_iter > 1 ? reinterpret_cast<float*>(ws + L.pf_base) : nullptr;
    a.part_pc = g.pf_max_iter > 1 ? reinterpret_cast<float*>(ws + L.part_pc) : nullptr;
    a.gscale = (float)(aniso ? 2.0 : 2.0 * p0.kappa);
    g.lap_valid = false;
    // one grain: its rotated table serves every voxel (no per-voxel rotation)
    const bool rotated = pg.grain_rot != nullptr;
    a.rot = (rotated && G > 1) ? reinterpret_cast<float*>(ws + L.rot) : nullptr;
    if (rotated && G > 1) {
      // crystal-frame table shared by every grain: [C 21][dC_q 21 x V][eps0_q 6 x V]
      pack_sym(pg.C_grain, a.xtab);
      for (int q = 0; q < nv; ++q) {
        double d[36];
        for (int i = 0; i < 36; ++i) d[i] = pg.C_var[36 * q + i] - pg.C_grain[i];
        pack_sym(d, a.xtab + 21 * (q + 1));
        for (int k = 0; k < 6; ++k) a.xtab[21 * (nv + 1) + 6 * q + k] = (float)pg.eps0[6 * q + k];
      }
    }
    a.spec = reinterpret_cast<float2*>(ws + L.spec);
    if (a.gid) {
      // every grain id must index the tables: block maxima of the field in
      // the spectral buffer (unused until the first transform), reduced here
      constexpr int kGidBlocks = 256;
      int gmax[kGidBlocks];
      int* dmax = reinterpret_cast<int*>(a.spec);
      if ((e = pfl::grain_id_max(a.gid, g.nvox, dmax, kGidBlocks, c->stream)) != hipSuccess ||
          (e = hipMemcpyAsync(gmax, dmax, sizeof(gmax), hipMemcpyDeviceToHost, c->stream)) != hipSuccess ||
          (e = hipStreamSynchronize(c->stream)) != hipSuccess)
        return bail(e, "grain id check");
      const int mx = *std::max_element(gmax, gmax + kGidBlocks);
      if (mx >= G) {
        fprintf(stderr, "pf_init: grain_id holds %d, not below n_grains = %d\n", mx, G);
        hipHostFree(c->host_status);
        hipHostFree(c->host_loads);
        delete c;
        return PF_EINVAL;
      }
    }
    float2* tw = reinterpret_cast<float2*>(ws + L.tw);
    a.tw_xh = tw;
    a.tw_x = tw + g.nx / 2;
    a.tw_y = tw + g.nx / 2 + g.nx;
    a.tw_z = tw + g.nx / 2 + g.nx + g.ny;
    a.part_ms = reinterpret_cast<double*>(ws + L.part_ms);
    a.part_res = reinterpret_cast<double*>(ws + L.part_res);
    a.part_ac = reinterpret_cast<double*>(ws + L.part_ac);
    a.part_mm = reinterpret_cast<float*>(ws + L.part_mm);
    a.part_gd = reinterpret_cast<double*>(ws + L.part_gd);
    a.state = reinterpret_cast<DevState*>(ws + L.state);
    a.pub = status_dev + status_off;
    g.status_off = status_off;
    status_off += g.ninst;
    a.save_stress = 0;

    // per-instance tables, stacked
    std::vector<float> tab, ref, kh, gk;
    std::vector<double> bss, khd;
    for (int m : g.members) {
      const InstanceHost& h = hosts[m];
      tab.insert(tab.end(), h.tab.begin(), h.tab.end());
      ref.insert(ref.end(), h.ref, h.ref + pft::kRefStride);
      kh.insert(kh.end(), h.kh, h.kh + pft::kKhStride);
      bss.insert(bss.end(), h.bss, h.bss + 36);
      khd.insert(khd.end(), h.khd, h.khd + pft::kKhdStride);
      gk.insert(gk.end(), h.gk, h.gk + pft::kGkStride);
    }
    std::vector<float> twh(2 * (size_t)(g.nx / 2 + g.nx + g.ny + g.nz));
    twiddles(g.nx / 2, twh.data());
    twiddles(g.nx, twh.data() + 2 * (g.nx / 2));
    twiddles(g.ny, twh.data() + 2 * (g.nx / 2 + g.nx));
    twiddles(g.nz, twh.data() + 2 * (g.nx / 2 + g.nx + g.ny));
    std::vector<DevState> st0(g.ninst);
    std::memset(st0.data(), 0, sizeof(DevState) * g.ninst);
    auto h2d = [&](const void* dst, const void* src, size_t bytes) {
      return hipMemcpyAsync(const_cast<void*>(dst), src, bytes, hipMemcpyHostToDevice, c->stream);
    };
    if ((e = h2d(a.tables, tab.data(), tab.size() * sizeof(float))) != hipSuccess) return bail(e, "tables");
    if (a.rot && (e = h2d(a.rot, hosts[g.members[0]].rot.data(), hosts[g.members[0]].rot.size() * sizeof(float))) !=
                     hipSuccess)
      return bail(e, "rotations");
    if ((e = h2d(a.ref, ref.data(), ref.size() * sizeof(float))) != hipSuccess) return bail(e, "reference");
    if ((e = h2d(a.kh, kh.data(), kh.size() * sizeof(float))) != hipSuccess) return bail(e, "spectral tables");
    if ((e = h2d(a.bss, bss.data(), bss.size() * sizeof(double))) != hipSuccess) return bail(e, "mixed condition");
    if ((e = h2d(a.khd, khd.data(), khd.size() * sizeof(double))) != hipSuccess) return bail(e, "spectral tables");
    if (a.gk && (e = h2d(a.gk, gk.data(), gk.size() * sizeof(float))) != hipSuccess)
      return bail(e, "gradient tables");
    if (a.krem && (e = h2d(a.krem, hosts[g.members[0]].krem.data(), hosts[g.members[0]].krem.size() * sizeof(float))) !=
                      hipSuccess)
      return bail(e, "per-grain gradient tables");
    if ((e = h2d(tw, twh.data(), twh.size() * sizeof(float))) != hipSuccess) return bail(e, "twiddles");
    if ((e = h2d(a.state, st0.data(), st0.size() * sizeof(DevState))) != hipSuccess) return bail(e, "state");
    // the host vectors above are pageable: the copies complete before return
    for (size_t j = 0; j < g.members.size(); ++j) {
      const pf_problem& pm = probs[g.members[j]];
      for (int q = 0; q < nv; ++q) {
        float* dst = a.eta + ((size_t)q * g.ninst + j) * g.nvox;
        if ((e = hipMemcpyAsync(dst, pm.eta0 + (size_t)q * g.nvox, sizeof(float) * g.nvox, hipMemcpyDeviceToDevice,
                                c->stream)) != hipSuccess)
          return bail(e, "eta0");
      }
    }
    if ((e = hipMemsetAsync(a.eps, 0, sizeof(float) * g.nvox * g.ninst * 6, c->stream)) != hipSuccess)
      return bail(e, "strain");
    if (g.own_epsp &&
        (e = hipMemsetAsync(ws + L.epsp, 0, sizeof(float) * g.nvox * g.ninst * 6, c->stream)) != hipSuccess)
      return bail(e, "plastic strain");
    // gradient energy of the initial state
    if ((e = pfl::raw_x_forward(a, a.eta, nv, c->stream)) != hipSuccess) return bail(e, "init x");
    if ((e = pfl::y_pass(a, nv, 1, c->stream)) != hipSuccess) return bail(e, "init y");
    if ((e = pfl::ac_z_update(a, 1, c->stream)) != hipSuccess) return bail(e, "init z");
    if ((e = pfl::ac_finalize(a, 1, c->stream)) != hipSuccess) return bail(e, "init fin");
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return bail(e, "init sync");
  }
  *out = c;
  return PF_OK;
}

int pf_init(const pf_problem* p, void* workspace, size_t ws_bytes, void* hip_stream, pf_ctx** out) {
  return pf_batch_init(p, 1, workspace, ws_bytes, hip_stream, out);
}

int pf_batch_step(pf_ctx* c, int32_t n_steps, const pf_load* loads) {
  if (!c) return PF_EINVAL;
  if (!loads || n_steps < 0) return fail(c, PF_EINVAL, "pf_step: bad arguments");
  uint32_t flags = 0;
  for (int i = 0; i < c->n_inst; ++i) flags |= loads[i].flags;
  const bool save_stress = (flags & PF_STEP_SAVE_STRESS) != 0;
  const bool force_fp = (flags & PF_STEP_FIXED_POINT) != 0;
  hipError_t e;
  // plastic strain: the caller's buffer in place for one instance, a copy
  // into the group's stacked field for a batch
  for (int i = 0; i < c->n_inst; ++i) {
    if (!loads[i].eps_p) continue;
    Group& g = c->groups[c->where[i].first];
    if (!g.own_epsp) {
      g.args.epsp = loads[i].eps_p;
    } else {
      float* stack = reinterpret_cast<float*>(c->ws + g.base + g.L.epsp);
      const int j = c->where[i].second;
      for (int comp = 0; comp < 6; ++comp) {
        e = hipMemcpyAsync(stack + ((size_t)comp * g.ninst + j) * g.nvox, loads[i].eps_p + (size_t)comp * g.nvox,
                           sizeof(float) * g.nvox, hipMemcpyDeviceToDevice, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "plastic strain copy");
      }
      g.args.epsp = stack;
    }
    g.epsp_given = true;
  }
  PF_TRY(upload_loads(c, loads));
  // path of each group
  std::vector<char> use_kh(c->groups.size());
  bool graphable = !save_stress && !c->prof_on && n_steps > 0;
  std::string key;
  for (size_t k = 0; k < c->groups.size(); ++k) {
    Group& g = c->groups[k];
    g.args.save_stress = save_stress ? 1 : 0;
    use_kh[k] = g.homogeneous && !g.epsp_given && !save_stress && !force_fp && !g.mobile && g.pf_max_iter <= 1;
    if (g.mobile && !g.lap_valid && n_steps > 0) {
      PF_TRY(refresh_gradient_force(c, g));
      g.lap_valid = true;
    }
    if (!use_kh[k] && (!g.one_iteration || g.pf_max_iter > 1)) graphable = false;
    char buf[64];
    snprintf(buf, sizeof(buf), "%d:%p;", (int)use_kh[k], (const void*)g.args.epsp);
    key += buf;
  }
  if (graphable) {
    PF_TRY(run_graph(c, n_steps, use_kh, key));
    for (size_t k = 0; k < c->groups.size(); ++k)
      if (!use_kh[k]) c->groups[k].fin_seq += n_steps;
    for (size_t k = 0; k < c->groups.size(); ++k) {
      Group& g = c->groups[k];
      if (use_kh[k]) {
        g.strain_valid = false;
        g.hist = 0;
      } else {
        g.strain_valid = true;
        g.hist += n_steps;
      }
    }
  } else {
    hipStream_t s = c->stream;
    for (int n = 0; n < n_steps; ++n) {
      // fixed-point groups that iterate: first iterate extrapolated from the
      // two previous steps (from the third step on), the step's starting
      // strain kept for that from the second step on
      std::vector<size_t> iterating;
      for (size_t k = 0; k < c->groups.size(); ++k)
        if (!use_kh[k] && !c->groups[k].one_iteration) iterating.push_back(k);
      // The first iterate extrapolates the converged strains of the previous
      // steps (linear from the third step on, quadratic from the fourth, cubic
      // from the fifth) and is written over the oldest of the four fields.
      std::vector<KArgs> first(c->groups.size()), later(c->groups.size());
      bool replay = !save_stress && !c->prof_on && !iterating.empty();
      int P = 1;  // iterations the replayed graph holds: those of the last step
      for (size_t k : iterating) {
        Group& g = c->groups[k];
        const int order = !g.strain_valid ? 0 : (g.hist >= 4 ? 3 : (g.hist == 3 ? 2 : (g.hist == 2 ? 1 : 0)));
        float* out = g.ring[(g.cur + 1) % 4];
        KArgs& f = first[k];
        f = g.args;
        f.skip_done = 1;
        f.eps = g.ring[g.cur];
        f.eps_out = out;
        f.eps_h1 = g.ring[(g.cur + 3) % 4];
        f.eps_h2 = g.ring[(g.cur + 2) % 4];
        f.eps_h3 = g.ring[(g.cur + 1) % 4];
        f.iter_mode = order;
        KArgs& l = later[k];
        l = g.args;
        l.skip_done = 1;
        l.eps = out;
        l.eps_out = out;
        l.eps_h1 = l.eps_h2 = l.eps_h3 = nullptr;
        l.iter_mode = 0;
        replay = replay && order == 3 && g.pf_max_iter <= 1;
        P = std::max(P, g.last_iters);
      }
      P = std::min(P, c->ms_max_iter);
      std::vector<size_t> active = iterating;
      std::vector<char> updated(c->groups.size(), 0);
      int it0 = 0;
      if (replay) {
        // The whole step as one graph: the fixed point runs P iterations on
        // the device (iterations after convergence exit at once), then each
        // group's update runs if all of its instances converged. One status
        // read per step; a group that needs more iterations continues here.
        std::string key = "P" + std::to_string(P);
        for (size_t k = 0; k < c->groups.size(); ++k) {
          char buf[80];
          snprintf(buf, sizeof(buf), ";%d:%d:%p", (int)use_kh[k], c->groups[k].cur,
                   (const void*)c->groups[k].args.epsp);
          key += buf;
        }
        PF_TRY(run_step_graph(c, key, [&](hipStream_t cs) -> int {
          for (size_t k = 0; k < c->groups.size(); ++k) {
            const Group& g = c->groups[k];
            if (use_kh[k] || g.one_iteration) {
              PF_TRY(fixed_step(c, g, use_kh[k] != 0, false, cs));
              continue;
            }
            PF_TRY(launch(c, cs, "step_begin", [&] { return pfl::step_begin(first[k], cs); }));
            PF_TRY(ms_iteration(c, first[k], cs));
            for (int it = 1; it < P; ++it) PF_TRY(ms_iteration(c, later[k], cs));
            PF_TRY(launch(c, cs, "group_ready", [&] { return pfl::group_ready(later[k], cs); }));
            KArgs ua = g.args;
            ua.eps = ua.eps_out = later[k].eps_out;
            ua.guard_ready = 1;
            PF_TRY(ac_update_args(c, g, ua, cs));
          }
          return PF_OK;
        }));
        if (n == n_steps - 1)
          for (size_t k = 0; k < c->groups.size(); ++k)
            if (use_kh[k]) PF_TRY(kh_finalize(c, c->groups[k], s));
        for (size_t k = 0; k < c->groups.size(); ++k)
          if (!use_kh[k]) c->groups[k].fin_seq += c->groups[k].one_iteration ? 1 : P;
        PF_TRY(wait_published(c, iterating));
        std::vector<size_t> still;
        for (size_t k : iterating) {
          const size_t b = status_base(c, k);
          bool all = true;
          for (int j = 0; j < c->groups[k].ninst; ++j) all = all && c->host_status[b + j].done;
          if (all) updated[k] = 1;
          else still.push_back(k);
        }
        active.swap(still);
        it0 = P;
        c->steps_replayed += 1;
      } else {
        for (size_t k = 0; k < c->groups.size(); ++k)
          if (use_kh[k] || c->groups[k].one_iteration) {
            PF_TRY(fixed_step(c, c->groups[k], use_kh[k] != 0, n == n_steps - 1, s));
            if (!use_kh[k]) c->groups[k].fin_seq += 1;
          }
        for (size_t k : iterating) PF_TRY(launch(c, s, "step_begin", [&] { return pfl::step_begin(first[k], s); }));
      }
      for (int it = it0; it < c->ms_max_iter && !active.empty(); ++it) {
        for (size_t k : active) {
          PF_TRY(ms_iteration(c, it == 0 ? first[k] : later[k], s));
          c->groups[k].fin_seq += 1;
        }
        PF_TRY(wait_published(c, active));
        std::vector<size_t> still;
        for (size_t k : active) {
          const size_t b = status_base(c, k);
          bool all = true;
          for (int j = 0; j < c->groups[k].ninst; ++j) all = all && c->host_status[b + j].done;
          if (!all) still.push_back(k);
        }
        active.swap(still);
      }
      if (!active.empty()) {
        const size_t k = active[0];
        const size_t b = status_base(c, k);
        double worst = 0.0;
        for (int j = 0; j < c->groups[k].ninst; ++j)
          if (!c->host_status[b + j].done && c->host_status[b + j].residual > worst)
            worst = c->host_status[b + j].residual;
        char buf[160];
        snprintf(buf, sizeof(buf), "fixed point not converged after %d iterations (residual %.3e)",
                 c->ms_max_iter, worst);
        for (size_t kk : iterating) c->groups[kk].hist = 0;
        return fail(c, PF_ENOCONV, buf);
      }
      for (size_t k : iterating) {
        const size_t b = status_base(c, k);
        for (int j = 0; j < c->groups[k].ninst; ++j)
          if (c->host_status[b + j].nonfinite) {
            for (size_t kk : iterating) c->groups[kk].hist = 0;
            return fail(c, PF_ENONFINITE,
                        "non-finite strain in the fixed point of instance " + std::to_string(c->groups[k].members[j]));
          }
      }
      for (size_t k : iterating) {
        Group& g = c->groups[k];
        const size_t b = status_base(c, k);
        int most = 0;
        for (int j = 0; j < g.ninst; ++j) most = std::max(most, (int)c->host_status[b + j].iters);
        g.last_iters = most;
        g.cur = (g.cur + 1) % 4;
        g.args.eps = g.args.eps_out = g.ring[g.cur];
        if (!updated[k]) PF_TRY(ac_update(c, g, s));
      }
      for (size_t k = 0; k < c->groups.size(); ++k) {
        Group& g = c->groups[k];
        if (use_kh[k]) {
          g.strain_valid = false;
          g.hist = 0;
        } else {
          g.strain_valid = true;
          g.hist += 1;
        }
      }
    }
  }
  c->steps += n_steps;
  if (n_steps > 0) {
    PF_TRY(read_status(c));
    size_t b = 0;
    for (auto& g : c->groups) {
      for (int j = 0; j < g.ninst; ++j)
        if (c->host_status[b + j].nonfinite)
          return fail(c, PF_ENONFINITE, "non-finite order parameter in instance " + std::to_string(g.members[j]));
      b += g.ninst;
    }
  }
  return PF_OK;
}

int pf_step(pf_ctx* c, int32_t n_steps, const pf_load* load) {
  if (!c) return PF_EINVAL;
  if (c->n_inst != 1) return fail(c, PF_EINVAL, "pf_step: batched context, use pf_batch_step");
  return pf_batch_step(c, n_steps, load);
}

int pf_batch_fields(pf_ctx* c, int32_t inst, int32_t which, int32_t set, float* buf) {
  if (!c) return PF_EINVAL;
  PF_TRY(check_instance(c, inst));
  if (!buf) return fail(c, PF_EINVAL, "pf_fields: null buffer");
  Group& g = c->groups[c->where[inst].first];
  const int j = c->where[inst].second;
  float* f = nullptr;
  int ncomp = 0;
  switch (which) {
    case PF_FIELD_ETA: f = g.args.eta; ncomp = c->nv; break;
    case PF_FIELD_STRAIN:
      if (!set && !g.strain_valid)
        return fail(c, PF_EINVAL,
                    "pf_fields: the homogeneous spectral path keeps no strain field; run the step with "
                    "PF_STEP_SAVE_STRESS or PF_STEP_FIXED_POINT");
      f = g.args.eps; ncomp = 6; break;
    case PF_FIELD_STRESS:
      if (set) return fail(c, PF_EINVAL, "pf_fields: stress is read-only");
      f = g.args.sig; ncomp = 6; break;
    default: return fail(c, PF_EINVAL, "pf_fields: unknown field");
  }
  if (set) {
    g.hist = 0;  // the strain history no longer describes the state
    if (which == PF_FIELD_STRAIN) g.strain_valid = true;
  }
  for (int comp = 0; comp < ncomp; ++comp) {
    float* slot = f + ((size_t)comp * g.ninst + j) * g.nvox;
    float* ext = buf + (size_t)comp * g.nvox;
    hipError_t e = set ? hipMemcpyAsync(slot, ext, g.nvox * sizeof(float), hipMemcpyDeviceToDevice, c->stream)
                       : hipMemcpyAsync(ext, slot, g.nvox * sizeof(float), hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "pf_fields");
  }
  if (set && which == PF_FIELD_ETA) {
    PF_TRY(refresh_gradient_energy(c, g));
    g.lap_valid = false;
  }
  if (set && which == PF_FIELD_STRAIN) {
    hipError_t e = pfl::strain_mean(g.args, f, j, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "pf_fields: strain mean");
  }
  return PF_OK;
}

int pf_fields(pf_ctx* c, int32_t which, int32_t set, float* buf) {
  if (!c) return PF_EINVAL;
  return pf_batch_fields(c, 0, which, set, buf);
}

int pf_batch_stats(pf_ctx* c, int32_t inst, pf_stats* out) {
  if (!c || !out) return PF_EINVAL;
  PF_TRY(check_instance(c, inst));
  const Group& g = c->groups[c->where[inst].first];
  DevState st;
  hipError_t e = hipMemcpyAsync(&st, g.args.state + c->where[inst].second, sizeof(DevState),
                                hipMemcpyDeviceToHost, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "stats copy");
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "stats sync");
  const double ntot = (double)g.nvox, dV = c->dx * c->dx * c->dx;
  std::memset(out, 0, sizeof(*out));
  out->step = c->steps;
  out->G_dw = g.args.A * st.stats[0] * dV;
  out->G_me = st.stats[1] * dV;
  for (int k = 0; k < 6; ++k) {
    out->sig_mean[k] = st.stats[2 + k] / ntot;
    out->eps_mean[k] = st.stats[8 + k] / ntot;
  }
  for (int q = 0; q < c->nv; ++q) out->eta_mean[q] = st.stats[14 + q] / ntot;
  // with gradient tables the sums already carry K (isotropic: kappa |xi|^2)
  out->G_gd = (g.args.gk ? 1.0 : c->kappa) * st.stats[pft::kQac] * dV / ntot;
  out->eta_min = st.stats[pft::kQac + 1];
  out->eta_max = st.stats[pft::kQac + 2];
  out->ms_iters = st.st.iters;
  out->ms_residual = st.st.residual;
  out->pf_iters = g.pf_max_iter > 1 ? st.st.pf_iters : 1;
  out->pf_change = g.pf_max_iter > 1 ? st.st.pf_change : 0.0;
  out->steps_replayed = c->steps_replayed;
  if (st.st.nonfinite) return fail(c, PF_ENONFINITE, "non-finite order parameter");
  return PF_OK;
}

int pf_stats_get(pf_ctx* c, pf_stats* out) {
  if (!c || !out) return PF_EINVAL;
  return pf_batch_stats(c, 0, out);
}

int pf_fft(pf_ctx* c, int32_t direction, int32_t ncomp, float* real, void* spec) {
  if (!c) return PF_EINVAL;
  if (c->n_inst != 1) return fail(c, PF_EUNSUPPORTED, "pf_fft: single-instance contexts only");
  if (!real || !spec || ncomp < 1 || ncomp > 6 || (direction != 1 && direction != -1))
    return fail(c, PF_EINVAL, "pf_fft: bad arguments");
  const Group& g = c->groups[0];
  KArgs a = g.args;
  a.spec = reinterpret_cast<float2*>(spec);
  // caller layout: unpadded rows of nx/2+1 coefficients, Nyquist in its row
  a.sh = a.ncol = g.nh;
  a.nq_row = 1;
  a.nqo = 0;
  a.cs = (size_t)g.nh * g.ny * g.nz;
  hipStream_t s = c->stream;
  if (direction == 1) {
    PF_TRY(launch(c, s, "fft_x_forward", [&] { return pfl::raw_x_forward(a, real, ncomp, s); }));
    PF_TRY(launch(c, s, "fft_y_forward", [&] { return pfl::y_pass(a, ncomp, 1, s); }));
    PF_TRY(launch(c, s, "fft_z_forward", [&] { return pfl::raw_z(a, ncomp, 1, s); }));
  } else {
    PF_TRY(launch(c, s, "fft_z_inverse", [&] { return pfl::raw_z(a, ncomp, -1, s); }));
    PF_TRY(launch(c, s, "fft_y_inverse", [&] { return pfl::y_pass(a, ncomp, -1, s); }));
    PF_TRY(launch(c, s, "fft_x_inverse",
                  [&] { return pfl::raw_x_inverse(a, real, ncomp, (float)(1.0 / (double)g.nvox), s); }));
  }
  return PF_OK;
}

// ---------------------------------------------------------------- autotuner
// Per size group, the launch plan of every column pass: for the y passes the
// FFT plan variant (radix split and elements per thread, 3 candidates) and
// the column tile (8 or 16 pencils per block); for the Green z pass of the
// fixed point the plan variant (2) and tile (8 or 16); for the Allen-Cahn z
// pass the plan variant (3); for the spectral path's z pass the plan variant
// (2) and tile (8 or 16). Candidates whose block would exceed 1024 threads
// are skipped. Each pass is timed within the passes a step runs around it, on
// the group's own fields and spectral buffer (zeroed first: it holds nothing
// between steps; no field of the state is written and the instances' FP64
// state is saved and restored); candidates alternate over two rounds and the
// best time counts. The choice is kept in the context and
// optionally cached as one JSON object per line.
}  // extern "C"

namespace {

struct TuneKey {
  char dev[128];
  int cus, nx, ny, nz, ninst, nv, spectral;
};

// candidate lists of the passes, in the order their times are written
struct Cand {
  int plan, tile;
};
constexpr Cand kYCand[6] = {{0, 8}, {0, 16}, {1, 8}, {1, 16}, {2, 8}, {2, 16}};
constexpr Cand kZmsCand[4] = {{0, 8}, {0, 16}, {1, 8}, {1, 16}};
constexpr Cand kZacCand[3] = {{0, 16}, {1, 16}, {2, 16}};
constexpr Cand kZkhCand[4] = {{0, 8}, {0, 16}, {1, 8}, {1, 16}};

// an entry as written, and the same fields as read back
const char* kTuneOut =
    "{\"device\":\"%s\",\"cus\":%d,\"nx\":%d,\"ny\":%d,\"nz\":%d,\"ninst\":%d,\"nv\":%d,"
    "\"spectral\":%d,\"ytile\":%d,\"yplan\":%d,\"ztile_ms\":%d,\"zplan_ms\":%d,\"zplan_ac\":%d,"
    "\"ztile_kh\":%d,\"zplan_kh\":%d";
const char* kTuneIn =
    "{\"device\":\"%127[^\"]\",\"cus\":%d,\"nx\":%d,\"ny\":%d,\"nz\":%d,\"ninst\":%d,\"nv\":%d,"
    "\"spectral\":%d,\"ytile\":%d,\"yplan\":%d,\"ztile_ms\":%d,\"zplan_ms\":%d,\"zplan_ac\":%d,"
    "\"ztile_kh\":%d,\"zplan_kh\":%d";

bool same_key(const TuneKey& a, const TuneKey& b) {
  return std::strcmp(a.dev, b.dev) == 0 && a.cus == b.cus && a.nx == b.nx && a.ny == b.ny && a.nz == b.nz &&
         a.ninst == b.ninst && a.nv == b.nv && a.spectral == b.spectral;
}

// a plan every pass of a group of this grid can launch
bool plan_valid(const pf_plan& p, int ny, int nz) {
  return pfl::plan_fits(0, ny, p.yplan, p.ytile) && pfl::plan_fits(1, nz, p.zplan_ms, p.ztile_ms) &&
         pfl::plan_fits(2, nz, p.zplan_ac, 16) && pfl::plan_fits(3, nz, p.zplan_kh, p.ztile_kh);
}

// last valid entry of the cache for key (entries are appended), or false
bool tune_cache_read(const char* path, const TuneKey& key, pf_plan& plan) {
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[4096];
  bool hit = false;
  while (std::fgets(line, sizeof(line), f)) {
    TuneKey k{};
    pf_plan p{};
    if (std::sscanf(line, kTuneIn, k.dev, &k.cus, &k.nx, &k.ny, &k.nz, &k.ninst, &k.nv, &k.spectral, &p.ytile,
                    &p.yplan, &p.ztile_ms, &p.zplan_ms, &p.zplan_ac, &p.ztile_kh, &p.zplan_kh) == 15 &&
        same_key(k, key) && plan_valid(p, key.ny, key.nz)) {
      plan = p;
      hit = true;
    }
  }
  std::fclose(f);
  return hit;
}

void write_times(FILE* f, const char* name, const double* us, int n) {
  std::fprintf(f, ",\"%s\":[", name);
  for (int i = 0; i < n; ++i) std::fprintf(f, i ? ",%.2f" : "%.2f", us[i] < 1e29 ? us[i] : -1.0);
  std::fprintf(f, "]");
}

// times: microseconds per candidate in the order of the lists above, -1 for
// candidates not timed (block too large, or a pass the group does not run)
bool tune_cache_append(const char* path, const TuneKey& k, const pf_plan& p, const double* us_y,
                       const double* us_zms, const double* us_zac, const double* us_zkh) {
  FILE* f = std::fopen(path, "a");
  if (!f) return false;
  std::fprintf(f, kTuneOut, k.dev, k.cus, k.nx, k.ny, k.nz, k.ninst, k.nv, k.spectral, p.ytile, p.yplan,
               p.ztile_ms, p.zplan_ms, p.zplan_ac, p.ztile_kh, p.zplan_kh);
  write_times(f, "us_y", us_y, 6);
  write_times(f, "us_zms", us_zms, 4);
  write_times(f, "us_zac", us_zac, 3);
  write_times(f, "us_zkh", us_zkh, 4);
  std::fprintf(f, "}\n");
  const bool ok = std::ferror(f) == 0;
  return std::fclose(f) == 0 && ok;
}

// average duration (us) of reps calls of f on stream s, after one warm-up call
template <class F>
int time_us(pf_ctx* c, hipStream_t s, int reps, F&& f, double& us) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = f();
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = f();
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(c, e, "autotune timing");
  us = 1e3 * ms / reps;
  return PF_OK;
}

// the plan a group launches with: its tuned or set one, else the defaults
pf_plan group_plan(const pf_ctx* c, const Group& g) {
  const KArgs& a = g.args;
  pf_plan p{};
  p.ytile = a.ytile ? a.ytile : 16;
  p.yplan = a.yplan;
  p.ztile_ms = a.ztile_ms ? a.ztile_ms : pft::kZmsTile;
  p.zplan_ms = a.zplan_ms;
  p.zplan_ac = a.zplan_ac;
  p.ztile_kh = a.ztile_kh ? a.ztile_kh : (c->nv == 1 ? 16 : 8);
  p.zplan_kh = a.zplan_kh;
  return p;
}

void apply_plan(Group& g, const pf_plan& p) {
  KArgs& a = g.args;
  a.ytile = p.ytile;
  a.yplan = p.yplan;
  a.ztile_ms = p.ztile_ms;
  a.zplan_ms = p.zplan_ms;
  a.zplan_ac = p.zplan_ac;
  a.ztile_kh = p.ztile_kh;
  a.zplan_kh = p.zplan_kh;
}

}  // namespace

extern "C" {

int pf_autotune(pf_ctx* c, const char* cache_path, uint32_t flags, int32_t* n_timed) {
  if (!c) return PF_EINVAL;
  if (c->capturing) return fail(c, PF_EINVAL, "pf_autotune: not during capture");
  hipStream_t s = c->stream;
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(c, e, "autotune sync");
  int dev = 0;
  hipDeviceProp_t prop;
  if ((e = hipGetDevice(&dev)) != hipSuccess || (e = hipGetDeviceProperties(&prop, dev)) != hipSuccess)
    return hip_fail(c, e, "autotune device");
  int timed = 0;
  constexpr int kReps = 10;
  for (auto& g : c->groups) {
    TuneKey key{};
    std::snprintf(key.dev, sizeof(key.dev), "%s", prop.gcnArchName);
    key.cus = prop.multiProcessorCount;
    key.nx = g.nx; key.ny = g.ny; key.nz = g.nz; key.ninst = g.ninst; key.nv = c->nv;
    key.spectral = (g.homogeneous && !g.mobile && g.pf_max_iter <= 1) ? 1 : 0;
    pf_plan plan = group_plan(c, g);
    if (cache_path && !(flags & PF_TUNE_RETIME) && tune_cache_read(cache_path, key, plan)) {
      apply_plan(g, plan);
      continue;
    }
    // the state of every instance is kept; during the timing no instance
    // counts as converged (the Green z pass skips converged instances)
    std::vector<DevState> saved(g.ninst);
    if ((e = hipMemcpyAsync(saved.data(), g.args.state, sizeof(DevState) * g.ninst, hipMemcpyDeviceToHost, s)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
      return hip_fail(c, e, "autotune setup");
    std::vector<DevState> live = saved;
    for (auto& st : live) st.st.done = 0;
    if ((e = hipMemcpyAsync(g.args.state, live.data(), sizeof(DevState) * g.ninst, hipMemcpyHostToDevice, s)) !=
            hipSuccess ||
        (e = hipMemsetAsync(g.args.spec, 0, g.L.spec_bytes, s)) != hipSuccess)
      return hip_fail(c, e, "autotune setup");
    double us_y[6], us_zms[4], us_zac[3], us_zkh[4];
    std::fill(us_y, us_y + 6, 1e30);
    std::fill(us_zms, us_zms + 4, 1e30);
    std::fill(us_zac, us_zac + 3, 1e30);
    std::fill(us_zkh, us_zkh + 4, 1e30);
    const int nv = c->nv;
    // Candidate k of a pass is timed inside the passes of one fixed-point
    // iteration (x forward, y forward, z, y inverse: the inverse x pass would
    // overwrite the strain), of one Allen-Cahn update or of one spectral
    // step, the other passes with the plan chosen so far (cur): timed alone,
    // the column passes ran at a different pace than after an x pass.
    // set(a, k) picks the candidate (false: it does not fit); best: the
    // fastest, -1 if none ran.
    KArgs cur = g.args;
    cur.skip_done = 0;
    int best = -1;
    auto tune_pass = [&](int ncand, double* us, auto&& set, auto&& run) -> int {
      for (int round = 0; round < 2; ++round)
        for (int k = 0; k < ncand; ++k) {
          KArgs a = cur;
          if (!set(a, k)) continue;
          double t = 0.0;
          PF_TRY(time_us(c, s, kReps, [&] { return run(a); }, t));
          us[k] = std::min(us[k], t);
        }
      best = -1;
      for (int k = 0; k < ncand; ++k)
        if (us[k] < 1e29 && (best < 0 || us[k] < us[best])) best = k;
      return PF_OK;
    };
    // the launches of a sequence stop at the first error
    auto chain = [](std::initializer_list<std::function<hipError_t()>> fs) {
      for (auto& f : fs) {
        const hipError_t r = f();
        if (r != hipSuccess) return r;
      }
      return hipSuccess;
    };
    auto fp_iteration = [&](const KArgs& xa, const KArgs& ya, const KArgs& za) {
      return chain({[&] { return pfl::ms_x_forward(xa, s); }, [&] { return pfl::y_pass(ya, 6, 1, s); },
                    [&] { return pfl::ms_z_green(za, s); }, [&] { return pfl::y_pass(ya, 6, -1, s); }});
    };
    auto ac_update = [&](const KArgs& ya, const KArgs& za) {
      return chain({[&] { return pfl::ac_x_forward(cur, s); }, [&] { return pfl::y_pass(ya, nv, 1, s); },
                    [&] { return pfl::ac_z_update(za, 0, s); }, [&] { return pfl::y_pass(ya, nv, -1, s); }});
    };
    auto kh_step = [&](const KArgs& ya, const KArgs& za) {
      return chain({[&] { return pfl::kh_x_forward(cur, 0, s); }, [&] { return pfl::y_pass(ya, 2 * nv, 1, s); },
                    [&] { return pfl::kh_z_update(za, 1, s); }, [&] { return pfl::y_pass(ya, nv, -1, s); }});
    };
    PF_TRY(tune_pass(6, us_y,
                     [&](KArgs& a, int k) {
                       a.yplan = kYCand[k].plan;
                       a.ytile = kYCand[k].tile;
                       return pfl::plan_fits(0, g.ny, a.yplan, a.ytile);
                     },
                     [&](const KArgs& a) { return key.spectral ? kh_step(a, cur) : fp_iteration(cur, a, cur); }));
    if (best < 0) return fail(c, PF_EDEVICE, "pf_autotune: no y-pass plan ran");
    plan.yplan = cur.yplan = kYCand[best].plan;
    plan.ytile = cur.ytile = kYCand[best].tile;
    if (!key.spectral) {
      PF_TRY(tune_pass(4, us_zms,
                       [&](KArgs& a, int k) {
                         a.zplan_ms = kZmsCand[k].plan;
                         a.ztile_ms = kZmsCand[k].tile;
                         return pfl::plan_fits(1, g.nz, a.zplan_ms, a.ztile_ms);
                       },
                       [&](const KArgs& a) { return fp_iteration(cur, cur, a); }));
      if (best < 0) return fail(c, PF_EDEVICE, "pf_autotune: no Green z-pass plan ran");
      plan.zplan_ms = cur.zplan_ms = kZmsCand[best].plan;
      plan.ztile_ms = cur.ztile_ms = kZmsCand[best].tile;
      PF_TRY(tune_pass(3, us_zac,
                       [&](KArgs& a, int k) {
                         a.zplan_ac = kZacCand[k].plan;
                         return pfl::plan_fits(2, g.nz, a.zplan_ac, 16);
                       },
                       [&](const KArgs& a) { return ac_update(cur, a); }));
      if (best < 0) return fail(c, PF_EDEVICE, "pf_autotune: no Allen-Cahn z-pass plan ran");
      plan.zplan_ac = cur.zplan_ac = kZacCand[best].plan;
    } else {
      PF_TRY(tune_pass(4, us_zkh,
                       [&](KArgs& a, int k) {
                         a.zplan_kh = kZkhCand[k].plan;
                         a.ztile_kh = kZkhCand[k].tile;
                         return pfl::plan_fits(3, g.nz, a.zplan_kh, a.ztile_kh);
                       },
                       [&](const KArgs& a) { return kh_step(cur, a); }));
      if (best < 0) return fail(c, PF_EDEVICE, "pf_autotune: no spectral z-pass plan ran");
      plan.zplan_kh = cur.zplan_kh = kZkhCand[best].plan;
      plan.ztile_kh = cur.ztile_kh = kZkhCand[best].tile;
    }
    if ((e = hipMemcpyAsync(g.args.state, saved.data(), sizeof(DevState) * g.ninst, hipMemcpyHostToDevice, s)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
      return hip_fail(c, e, "autotune restore");
    apply_plan(g, plan);
    ++timed;
    if (cache_path && !tune_cache_append(cache_path, key, plan, us_y, us_zms, us_zac, us_zkh))
      return fail(c, PF_EINVAL, std::string("pf_autotune: cannot write the cache ") + cache_path);
  }
  drop_graph(c);  // launches of a captured step carry the old plans
  if (n_timed) *n_timed = timed;
  return PF_OK;
}

int pf_batch_plan(pf_ctx* c, int32_t inst, pf_plan* out) {
  if (!c || !out) return PF_EINVAL;
  PF_TRY(check_instance(c, inst));
  *out = group_plan(c, c->groups[c->where[inst].first]);
  return PF_OK;
}

int pf_batch_set_plan(pf_ctx* c, int32_t inst, const pf_plan* plan) {
  if (!c || !plan) return PF_EINVAL;
  if (c->capturing) return fail(c, PF_EINVAL, "pf_batch_set_plan: not during capture");
  PF_TRY(check_instance(c, inst));
  Group& g = c->groups[c->where[inst].first];
  if (!plan_valid(*plan, g.ny, g.nz)) return fail(c, PF_EINVAL, "pf_batch_set_plan: no such plan for this grid");
  apply_plan(g, *plan);
  drop_graph(c);
  return PF_OK;
}

int pf_fft_plan(int32_t n, int32_t variant, int32_t* elems_per_thread, int32_t* radices, int32_t* n_stages) {
  if (!elems_per_thread || !radices || !n_stages || !pfl::supported_axis(n)) return PF_EINVAL;
  int e = 0, r[8];
  const int ns = pfl::plan_radices(n, variant, &e, r);
  if (ns == 0) return PF_EINVAL;
  *elems_per_thread = e;
  *n_stages = ns;
  for (int i = 0; i < ns; ++i) radices[i] = r[i];
  return PF_OK;
}

int pf_profile_enable(pf_ctx* c, int32_t on) {
  if (!c) return PF_EINVAL;
  hipStreamSynchronize(c->stream);
  for (auto& pe : c->prof) {
    c->ev_pool.push_back(pe.start);
    c->ev_pool.push_back(pe.stop);
  }
  c->prof.clear();
  c->prof_names.clear();
  c->prof_counts.clear();
  c->prof_ms.clear();
  c->prof_on = on != 0;
  return PF_OK;
}

int pf_profile_select(pf_ctx* c, const char* name) {
  if (!c) return PF_EINVAL;
  c->prof_only = name ? name : "";
  return PF_OK;
}

int pf_profile_read(pf_ctx* c, int32_t max_n, char (*names)[64], int64_t* counts, double* total_ms,
                    int32_t* n) {
  if (!c || !n) return PF_EINVAL;
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "profile sync");
  for (auto& pe : c->prof) {
    float ms = 0.f;
    hipEventElapsedTime(&ms, pe.start, pe.stop);
    size_t i = 0;
    while (i < c->prof_names.size() && c->prof_names[i] != pe.name) ++i;
    if (i == c->prof_names.size()) {
      c->prof_names.push_back(pe.name);
      c->prof_counts.push_back(0);
      c->prof_ms.push_back(0.0);
    }
    c->prof_counts[i] += 1;
    c->prof_ms[i] += ms;
    c->ev_pool.push_back(pe.start);
    c->ev_pool.push_back(pe.stop);
  }
  c->prof.clear();
  const int cnt = (int)c->prof_names.size();
  *n = cnt;
  for (int i = 0; i < cnt && i < max_n; ++i) {
    if (names) {
      std::strncpy(names[i], c->prof_names[i].c_str(), 63);
      names[i][63] = 0;
    }
    if (counts) counts[i] = c->prof_counts[i];
    if (total_ms) total_ms[i] = c->prof_ms[i];
  }
  return PF_OK;
}

int pf_destroy(pf_ctx* c) {
  if (!c) return PF_EINVAL;
  hipStreamSynchronize(c->stream);
  drop_graph(c);
  if (c->cap_stream) hipStreamDestroy(c->cap_stream);
  for (auto& pe : c->prof) {
    hipEventDestroy(pe.start);
    hipEventDestroy(pe.stop);
  }
  for (auto ev : c->ev_pool) hipEventDestroy(ev);
  if (c->host_status) hipHostFree(c->host_status);
  if (c->host_loads) hipHostFree(c->host_loads);
  delete c;
  return PF_OK;
}

const char* pf_last_error(const pf_ctx* c) {
  if (!c) return "null context";
  return c->err.c_str();
}

int pf_batch_size(const pf_ctx* c) { return c ? c->n_inst : 0; }

// ---------------------------------------------------------------- surrogate
int pf_macro_residual(pf_ctx* c, const float* eta_prev, int32_t n_steps, const pf_load* load, double* rho) {
  if (!c) return PF_EINVAL;
  if (!eta_prev || !load || !rho || n_steps < 1) return fail(c, PF_EINVAL, "pf_macro_residual: bad arguments");
  if (c->n_inst != 1) return fail(c, PF_EUNSUPPORTED, "pf_macro_residual: single-instance contexts only");
  Group& g = c->groups[0];
  if (!g.homogeneous || g.epsp_given || g.mobile)
    return fail(c, PF_EUNSUPPORTED,
                "pf_macro_residual: needs one stiffness, linear h, n_var <= 3, no plastic strain, uniform mobility");
  PF_TRY(upload_loads(c, load));
  const KArgs& a = g.args;
  hipStream_t s = c->stream;
  PF_TRY(launch(c, s, "res_x_forward", [&] { return pfl::ct_x_forward(a, eta_prev, n_steps, s); }));
  PF_TRY(launch(c, s, "res_y_forward", [&] { return pfl::y_pass(a, 3 * a.nv, 1, s); }));
  PF_TRY(launch(c, s, "res_z", [&] { return pfl::kh_z_update(a, 2, s); }));
  PF_TRY(launch(c, s, "res_y_inverse", [&] { return pfl::y_pass(a, a.nv, -1, s); }));
  PF_TRY(launch(c, s, "res_x_inverse", [&] { return pfl::kh_residual(a, eta_prev, n_steps, s); }));
  double r = 0.0;
  hipError_t e = hipMemcpyAsync(&r, &a.state->resid_max, sizeof(double), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return hip_fail(c, e, "residual copy");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(c, e, "residual sync");
  *rho = r;
  return PF_OK;
}

}  // extern "C"

struct pf_fno {
  pf_ctx* ctx;
  pfn::FArgs fa;
  std::vector<float> P, p;   // lift weights kept on the host (the constant part is folded per call)
  float* eta_prev;
  float* eta_pred;
};

namespace {

struct FnoLayout {
  size_t va, vb, x1, y1, x2, y2, tw, xt, W, b, R, Q1, q1, Q2, prev, pred, total;
};

FnoLayout fno_layout(int nx, int ny, int nz, int m) {
  FnoLayout L{};
  const size_t nvox = (size_t)nx * ny * nz;
  const size_t x1 = (size_t)nz * ny * m * 2 * pfn::kC, x2 = (size_t)nz * 2 * m * m * 2 * pfn::kC;
  const size_t rl = (size_t)(2 * m) * (2 * m) * m * pfn::kC * pfn::kC * 2;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
  L.va = take(nvox * pfn::kC * 2);
  L.vb = take(nvox * pfn::kC * 2);
  L.x1 = take(x1 * 4);
  L.y1 = take(x1 * 4);
  L.x2 = take(x2 * 4);
  L.y2 = take(x2 * 4);
  L.tw = take((size_t)(ny + nz) * 8);
  L.xt = take((size_t)2 * 2 * 32 * nx * 2);
  L.W = take((size_t)pfn::kLayers * pfn::kC * pfn::kC * 2);
  L.b = take((size_t)pfn::kLayers * pfn::kC * 4);
  L.R = take((size_t)pfn::kLayers * rl * 2);
  L.Q1 = take((size_t)pfn::kH * pfn::kC * 2);
  L.q1 = take((size_t)pfn::kH * 4);
  L.Q2 = take((size_t)pfn::kH * 4);
  L.prev = take(nvox * 4);
  L.pred = take(nvox * 4);
  L.total = off;
  return L;
}

uint16_t host_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// w ~ hi + lo with both parts BF16 (relative error about 2^-17)
void split_bf16(double w, uint16_t* hi, uint16_t* lo) {
  *hi = host_bf16((float)w);
  const uint32_t u = (uint32_t)*hi << 16;
  float h;
  std::memcpy(&h, &u, 4);
  *lo = host_bf16((float)(w - (double)h));
}

int fno_check(const pf_ctx* c, int32_t modes, std::string& why) {
  if (!c) { why = "null context"; return PF_EINVAL; }
  if (c->n_inst != 1) { why = "single-instance contexts only"; return PF_EUNSUPPORTED; }
  const Group& g = c->groups[0];
  if (c->nv != 1) { why = "one order parameter only"; return PF_EUNSUPPORTED; }
  if (g.nx % 32 != 0 || g.nx > 128 || g.ny > 128 || g.nz > 128) {
    why = "grid: nx a multiple of 32, every axis <= 128";
    return PF_EUNSUPPORTED;
  }
  if (modes < 1 || modes > pfn::kMaxModes || 2 * modes > g.ny || 2 * modes > g.nz || modes > g.nx / 2) {
    why = "modes must be in 1..16 with 2 modes <= ny, nz and modes <= nx / 2";
    return PF_EINVAL;
  }
  return PF_OK;
}

}  // namespace

extern "C" {

int pf_fno_workspace_size(const pf_ctx* c, int32_t modes, size_t* bytes) {
  std::string why;
  if (!bytes) return PF_EINVAL;
  const int rc = fno_check(c, modes, why);
  if (rc != PF_OK) return rc;
  const Group& g = c->groups[0];
  *bytes = fno_layout(g.nx, g.ny, g.nz, modes).total;
  return PF_OK;
}

int pf_fno_init(pf_ctx* c, const pf_fno_weights* w, void* workspace, size_t ws_bytes, pf_fno** out) {
  if (!c || !out) return PF_EINVAL;
  *out = nullptr;
  std::string why;
  if (!w) return fail(c, PF_EINVAL, "pf_fno_init: null weights");
  if (w->width != pfn::kC || w->hidden != pfn::kH || w->n_layers != pfn::kLayers || w->n_cond != pfn::kCond)
    return fail(c, PF_EUNSUPPORTED, "pf_fno_init: this build supports width 32, hidden 128, 4 layers, 7 "
                                    "conditioning channels");
  int rc = fno_check(c, w->modes, why);
  if (rc != PF_OK) return fail(c, rc, "pf_fno_init: " + why);
  if (!w->P || !w->p || !w->W || !w->b || !w->R || !w->Q1 || !w->q1 || !w->Q2)
    return fail(c, PF_EINVAL, "pf_fno_init: missing weights");
  const Group& g = c->groups[0];
  const int m = w->modes;
  const FnoLayout L = fno_layout(g.nx, g.ny, g.nz, m);
  if (!workspace || ws_bytes < L.total) return fail(c, PF_ENOMEM, "pf_fno_init: workspace too small");
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0)
    return fail(c, PF_EINVAL, "pf_fno_init: workspace must be 256-byte aligned");
  pf_fno* f = new (std::nothrow) pf_fno();
  if (!f) return PF_ENOMEM;
  char* ws = static_cast<char*>(workspace);
  pfn::FArgs& a = f->fa;
  std::memset(&a, 0, sizeof(a));
  a.nx = g.nx; a.ny = g.ny; a.nz = g.nz; a.m = m;
  a.nvox = g.nvox;
  a.inv_ntot = (float)(1.0 / (double)g.nvox);
  a.va = reinterpret_cast<uint16_t*>(ws + L.va);
  a.vb = reinterpret_cast<uint16_t*>(ws + L.vb);
  a.X1 = reinterpret_cast<float*>(ws + L.x1);
  a.Y1 = reinterpret_cast<float*>(ws + L.y1);
  a.X2 = reinterpret_cast<float*>(ws + L.x2);
  a.Y2 = reinterpret_cast<float*>(ws + L.y2);
  float2* tw = reinterpret_cast<float2*>(ws + L.tw);
  a.twy = tw;
  a.twz = tw + g.ny;
  uint16_t* xt = reinterpret_cast<uint16_t*>(ws + L.xt);
  a.wxf = xt;
  a.wxi = xt + (size_t)2 * 32 * g.nx;
  a.W = reinterpret_cast<uint16_t*>(ws + L.W);
  a.b = reinterpret_cast<float*>(ws + L.b);
  a.R = reinterpret_cast<uint16_t*>(ws + L.R);
  a.r_stride = (size_t)(2 * m) * (2 * m) * m * pfn::kC * pfn::kC * 2;
  a.Q1 = reinterpret_cast<uint16_t*>(ws + L.Q1);
  a.q1 = reinterpret_cast<float*>(ws + L.q1);
  a.Q2 = reinterpret_cast<float*>(ws + L.Q2);
  a.q2 = w->q2;
  f->eta_prev = reinterpret_cast<float*>(ws + L.prev);
  f->eta_pred = reinterpret_cast<float*>(ws + L.pred);
  f->ctx = c;
  f->P.assign(w->P, w->P + pfn::kC * (1 + pfn::kCond));
  f->p.assign(w->p, w->p + pfn::kC);
  // host conversions: BF16 weights, R reordered to [l][kz'][ky'][kx][o][i][re, im]
  const int C = pfn::kC, my = 2 * m;
  std::vector<float> twh(2 * (size_t)(g.ny + g.nz));
  twiddles(g.ny, twh.data());
  twiddles(g.nz, twh.data() + 2 * g.ny);
  // the x sums' matrices: row j = 2 kx + (re, im) of the forward sum, column j
  // of the inverse (1/N and the doubling of kx > 0 folded in), as BF16 hi and
  // lo parts of the double values
  std::vector<uint16_t> wx((size_t)4 * 32 * g.nx, 0);
  uint16_t* wxf = wx.data();
  uint16_t* wxi = wx.data() + (size_t)2 * 32 * g.nx;
  const double two_pi = 6.283185307179586476925286766559;
  for (int kx = 0; kx < m; ++kx)
    for (int x = 0; x < g.nx; ++x) {
      const double th = two_pi * (double)(((long long)kx * x) % g.nx) / g.nx;
      const double scale = (kx == 0 ? 1.0 : 2.0) / (double)g.nvox;
      const double f[2] = {std::cos(th), -std::sin(th)};
      for (int ri = 0; ri < 2; ++ri) {
        const int j = 2 * kx + ri;
        split_bf16(f[ri], &wxf[(size_t)j * g.nx + x], &wxf[(size_t)(32 + j) * g.nx + x]);
        split_bf16(scale * f[ri], &wxi[(size_t)x * 32 + j], &wxi[(size_t)(g.nx + x) * 32 + j]);
      }
    }
  std::vector<uint16_t> Wb((size_t)pfn::kLayers * C * C), Q1b((size_t)pfn::kH * C);
  for (size_t i = 0; i < Wb.size(); ++i) Wb[i] = host_bf16(w->W[i]);
  for (size_t i = 0; i < Q1b.size(); ++i) Q1b[i] = host_bf16(w->Q1[i]);
  std::vector<uint16_t> Rb((size_t)pfn::kLayers * a.r_stride);
  for (int l = 0; l < pfn::kLayers; ++l)
    for (int o = 0; o < C; ++o)
      for (int i = 0; i < C; ++i)
        for (int kz = 0; kz < my; ++kz)
          for (int ky = 0; ky < my; ++ky)
            for (int kx = 0; kx < m; ++kx) {
              const size_t src = ((((((size_t)l * C + o) * C + i) * my + kz) * my + ky) * m + kx) * 2;
              const size_t dst = (size_t)l * a.r_stride + (((((size_t)kz * my + ky) * m + kx) * C + o) * C + i) * 2;
              Rb[dst] = host_bf16(w->R[src]);
              Rb[dst + 1] = host_bf16(w->R[src + 1]);
            }
  hipError_t e;
  auto h2d = [&](const void* dst, const void* src, size_t bytes) {
    return hipMemcpyAsync(const_cast<void*>(dst), src, bytes, hipMemcpyHostToDevice, c->stream);
  };
  if ((e = h2d(tw, twh.data(), twh.size() * 4)) != hipSuccess || (e = h2d(xt, wx.data(), wx.size() * 2)) != hipSuccess ||
      (e = h2d(a.W, Wb.data(), Wb.size() * 2)) != hipSuccess ||
      (e = h2d(a.b, w->b, (size_t)pfn::kLayers * C * 4)) != hipSuccess ||
      (e = h2d(a.R, Rb.data(), Rb.size() * 2)) != hipSuccess || (e = h2d(a.Q1, Q1b.data(), Q1b.size() * 2)) != hipSuccess ||
      (e = h2d(a.q1, w->q1, pfn::kH * 4)) != hipSuccess || (e = h2d(a.Q2, w->Q2, pfn::kH * 4)) != hipSuccess ||
      (e = hipStreamSynchronize(c->stream)) != hipSuccess) {
    delete f;
    return hip_fail(c, e, "pf_fno_init upload");
  }
  *out = f;
  return PF_OK;
}

int pf_fno_forward(pf_fno* f, const double* cond, const float* eta_in, float* eta_out) {
  if (!f) return PF_EINVAL;
  pf_ctx* c = f->ctx;
  if (!cond || !eta_in || !eta_out || eta_in == eta_out) return fail(c, PF_EINVAL, "pf_fno_forward: bad arguments");
  pfn::FArgs a = f->fa;
  const int C = pfn::kC, ni = 1 + pfn::kCond;
  for (int o = 0; o < C; ++o) {
    double k = f->p[o];
    for (int j = 0; j < pfn::kCond; ++j) k += (double)f->P[o * ni + 1 + j] * cond[j];
    a.lift[o] = f->P[o * ni];
    a.lift[C + o] = (float)k;
  }
  hipStream_t s = c->stream;
  return launch(c, s, "fno_forward", [&] { return pfn::forward(a, eta_in, eta_out, s); });
}

int pf_fno_advance(pf_fno* f, int32_t n_calls, int32_t steps_per_call, const double* cond, const pf_load* load,
                   double tol, pf_fno_report* rep) {
  if (!f) return PF_EINVAL;
  pf_ctx* c = f->ctx;
  if (!cond || !load || !rep || n_calls < 0 || steps_per_call < 1)
    return fail(c, PF_EINVAL, "pf_fno_advance: bad arguments");
  Group& g = c->groups[0];
  float* eta = g.args.eta;
  const size_t bytes = sizeof(float) * g.nvox;
  hipStream_t s = c->stream;
  for (int n = 0; n < n_calls; ++n) {
    hipError_t e = hipMemcpyAsync(f->eta_prev, eta, bytes, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(c, e, "pf_fno_advance copy");
    PF_TRY(pf_fno_forward(f, cond, f->eta_prev, eta));
    double rho = 0.0;
    PF_TRY(pf_macro_residual(c, f->eta_prev, steps_per_call, load, &rho));
    rep->last_rho = rho;
    if (rho <= tol) {
      rep->accepted += 1;
      if (rho > rep->rho_max_accepted) rep->rho_max_accepted = rho;
      c->steps += steps_per_call;
      g.hist = 0;
      g.strain_valid = false;
      g.lap_valid = false;
      PF_TRY(refresh_gradient_energy(c, g));
    } else {
      rep->rejected += 1;
      if (rep->rho_min_rejected == 0.0 || rho < rep->rho_min_rejected) rep->rho_min_rejected = rho;
      e = hipMemcpyAsync(eta, f->eta_prev, bytes, hipMemcpyDeviceToDevice, s);
      if (e != hipSuccess) return hip_fail(c, e, "pf_fno_advance copy");
      PF_TRY(refresh_gradient_energy(c, g));
      PF_TRY(pf_batch_step(c, steps_per_call, load));
    }
  }
  return PF_OK;
}

int pf_fno_destroy(pf_fno* f) {
  if (!f) return PF_EINVAL;
  hipStreamSynchronize(f->ctx->stream);
  delete f;
  return PF_OK;
}

}  // extern "C"
