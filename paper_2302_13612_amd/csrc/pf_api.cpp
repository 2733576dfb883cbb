// Host runtime and C ABI of the phase-field twin step (see include/pf.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/pf.h"
#include "pf_device.hpp"

void pf_rotate_voigt(const double* Cv, const double* R9, double* out);  // pf_crystal.cpp

using pft::DevState;
using pft::KArgs;
using pft::Status;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

// Workspace layout (byte offsets from the workspace base).
struct Layout {
  size_t eta, eps, eps_prev, sig, spec, tables, rot, tw, part_ms, part_res, part_ac, part_mm, part_gd, state, total;
  int tab_stride;
};

int tab_stride_for(int nv) { return 21 * (nv + 1) + 6 * nv; }

bool axis_ok(int n) { return pfl::supported_axis(n); }

// Spectral rows of nx/2+1 coefficients are padded to a multiple of 16
// complex values (128 bytes) so every 16-column tile of the y and z passes is
// one aligned cache line per row.
int spec_stride(int nx) { return (nx / 2 + 1 + 15) / 16 * 16; }

Layout make_layout(int nx, int ny, int nz, int nv, int n_grains) {
  Layout L{};
  const size_t nvox = (size_t)nx * ny * nz;
  const size_t nh = (size_t)nx / 2 + 1;
  const size_t nspec = (size_t)spec_stride(nx) * ny * nz;
  KArgs a{};
  a.nx = nx; a.ny = ny; a.nz = nz; a.nh = (int)nh; a.sh = spec_stride(nx); a.nv = nv;
  const size_t xb = (size_t)pfl::x_blocks(a);
  const size_t zb = (size_t)pfl::z_blocks(a, nv > 6 ? nv : 6);
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
  L.eta = take(sizeof(float) * nvox * nv);
  L.eps = take(sizeof(float) * nvox * 6);
  L.eps_prev = take(sizeof(float) * nvox * 6);
  L.sig = take(sizeof(float) * nvox * 6);
  L.spec = take(sizeof(float) * 2 * nspec * 6);
  L.tab_stride = tab_stride_for(nv);
  L.tables = take(sizeof(float) * (size_t)L.tab_stride * (n_grains > 0 ? n_grains : 1));
  L.rot = take(sizeof(float) * 12 * (size_t)(n_grains > 0 ? n_grains : 1));
  L.tw = take(sizeof(float) * 2 * (size_t)(nx / 2 + nx + ny + nz));
  L.part_ms = take(sizeof(double) * xb * pft::kQms);
  L.part_res = take(sizeof(double) * xb * pft::kQres);
  L.part_ac = take(sizeof(double) * xb * pft::kQac);
  L.part_mm = take(sizeof(float) * xb * 2);
  L.part_gd = take(sizeof(double) * zb * pft::kQgd);
  L.state = take(sizeof(DevState));
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

// W_N^n = exp(-2 pi i n / N), computed in double, rounded once.
void twiddles(int N, float* out) {
  for (int n = 0; n < N; ++n) {
    const double ang = -2.0 * M_PI * (double)n / (double)N;
    out[2 * n] = (float)std::cos(ang);
    out[2 * n + 1] = (float)std::sin(ang);
  }
}

struct ProfEntry {
  std::string name;
  hipEvent_t start, stop;
};

}  // namespace

struct pf_ctx {
  int nx, ny, nz, nh, nv;
  size_t nvox;
  double dx, kappa;
  hipStream_t stream;
  char* ws;
  Layout L;
  KArgs args;
  bool one_iteration;
  int ms_max_iter;
  int64_t steps;
  int64_t hist;         // consecutive steps whose strain history is valid
  Status* host_status;  // pinned
  std::string err;
  bool prof_on;
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
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Launch one stage, bracketed by events when profiling is on.
template <class F>
int launch(pf_ctx* c, const char* name, F&& f) {
  ProfEntry pe;
  if (c->prof_on) {
    pe.name = name;
    pe.start = get_event(c);
    pe.stop = get_event(c);
    if (pe.start) hipEventRecord(pe.start, c->stream);
  }
  hipError_t e = f();
  if (e != hipSuccess) return hip_fail(c, e, name);
  if (c->prof_on && pe.start && pe.stop) {
    hipEventRecord(pe.stop, c->stream);
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
    why = "grid sizes must each be one of 32, 48, 64, 96, 128, 256";
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
  if (p->bc_stress_mask > 63u) { why = "bc_stress_mask has bits above 5"; return PF_EINVAL; }
  return PF_OK;
}

}  // namespace

extern "C" {

int pf_workspace_size(const pf_problem* p, size_t* bytes) {
  std::string why;
  if (!bytes) return PF_EINVAL;
  if (!p || !axis_ok(p->nx) || !axis_ok(p->ny) || !axis_ok(p->nz) || p->n_var < 1 ||
      p->n_var > pft::kMaxVar || p->n_grains < 1 || p->n_grains > 255)
    return PF_EINVAL;
  *bytes = make_layout(p->nx, p->ny, p->nz, p->n_var, p->n_grains).total;
  return PF_OK;
}

int pf_init(const pf_problem* p, void* workspace, size_t ws_bytes, void* hip_stream, pf_ctx** out) {
  if (!out) return PF_EINVAL;
  *out = nullptr;
  std::string why;
  int rc = validate(p, why);
  if (rc != PF_OK) {
    fprintf(stderr, "pf_init: %s\n", why.c_str());
    return rc;
  }
  const Layout L = make_layout(p->nx, p->ny, p->nz, p->n_var, p->n_grains);
  if (!workspace || ws_bytes < L.total) {
    fprintf(stderr, "pf_init: workspace of %zu bytes needed\n", L.total);
    return PF_ENOMEM;
  }
  if (reinterpret_cast<uintptr_t>(workspace) % kAlign != 0) {
    fprintf(stderr, "pf_init: workspace must be 256-byte aligned\n");
    return PF_EINVAL;
  }
  pf_ctx* c = new (std::nothrow) pf_ctx();
  if (!c) return PF_ENOMEM;
  c->nx = p->nx; c->ny = p->ny; c->nz = p->nz; c->nh = p->nx / 2 + 1; c->nv = p->n_var;
  c->nvox = (size_t)p->nx * p->ny * p->nz;
  c->dx = p->dx;
  c->kappa = p->kappa;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  c->ws = static_cast<char*>(workspace);
  c->L = L;
  c->steps = 0;
  c->hist = 0;
  c->prof_on = false;
  c->ms_max_iter = p->ms_max_iter;

  // material tables: per-grain sample-frame tables (rotated from the shared
  // crystal-frame material when rotations are given)
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
  std::vector<float> tab((size_t)L.tab_stride * G, 0.f);
  for (int g = 0; g < G; ++g) {
    float* t = tab.data() + (size_t)g * L.tab_stride;
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
  std::vector<float> rot((size_t)12 * G, 0.f);
  if (rotated)
    for (int g = 0; g < G; ++g)
      for (int k = 0; k < 9; ++k) rot[12 * g + k] = (float)p->grain_rot[9 * g + k];
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
  // one stiffness everywhere equal to the reference: the fixed point is exact
  // after one iteration.
  bool one = (G == 1);
  for (int i = 0; i < 36 && one; ++i) {
    if (Cg_s[i] != C0[i]) one = false;
    for (int q = 0; q < nv && one; ++q)
      if (Cv_s[36 * q + i] != Cg_s[i]) one = false;
  }
  c->one_iteration = one;

  // kernel arguments
  KArgs& a = c->args;
  std::memset(&a, 0, sizeof(a));
  a.nx = p->nx; a.ny = p->ny; a.nz = p->nz; a.nh = c->nh; a.sh = spec_stride(p->nx); a.nv = nv;
  a.h_kind = p->h_kind;
  a.n_grains = G;
  a.tab_stride = L.tab_stride;
  a.A = (float)p->A;
  a.LDt = (float)(p->L * p->dt);
  const double twopi = 2.0 * M_PI;
  const double kx = twopi / (p->nx * p->dx), ky = twopi / (p->ny * p->dx), kz = twopi / (p->nz * p->dx);
  const double f = 2.0 * p->L * p->dt * p->kappa;
  a.ax = (float)(f * kx * kx); a.ay = (float)(f * ky * ky); a.az = (float)(f * kz * kz);
  a.gx = kx * kx; a.gy = ky * ky; a.gz = kz * kz;
  a.inv_ntot = (float)(1.0 / (double)c->nvox);
  a.tol = p->ms_tol;
  pack_sym(C0, a.C0);
  double M0[36], S0[36];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) M0[6 * i + j] = 0.5 * (C0[6 * i + j] + C0[6 * j + i]) * (j < 3 ? 1.0 : 2.0);
  if (!invert(6, M0, S0)) {
    delete c;
    fprintf(stderr, "pf_init: reference stiffness is singular\n");
    return PF_EINVAL;
  }
  for (int i = 0; i < 36; ++i) a.S0[i] = (float)S0[i];
  a.stress_mask = p->bc_stress_mask;
  {
    int idx[6], ns = 0;
    for (int i = 0; i < 6; ++i)
      if ((p->bc_stress_mask >> i) & 1u) idx[ns++] = i;
    for (int i = 0; i < 36; ++i) a.Bss[i] = 0.0;
    if (ns > 0) {
      double sub[36], inv[36];
      for (int i = 0; i < ns; ++i)
        for (int j = 0; j < ns; ++j) sub[i * ns + j] = M0[6 * idx[i] + idx[j]];
      if (!invert(ns, sub, inv)) {
        delete c;
        fprintf(stderr, "pf_init: stress-controlled block of the reference stiffness is singular\n");
        return PF_EINVAL;
      }
      for (int i = 0; i < ns; ++i)
        for (int j = 0; j < ns; ++j) a.Bss[6 * idx[i] + idx[j]] = inv[i * ns + j];
    }
  }
  char* ws = c->ws;
  a.eta = reinterpret_cast<float*>(ws + L.eta);
  a.eps = reinterpret_cast<float*>(ws + L.eps);
  a.eps_prev = reinterpret_cast<float*>(ws + L.eps_prev);
  a.iter_mode = 0;
  a.sig = reinterpret_cast<float*>(ws + L.sig);
  a.epsp = nullptr;
  a.gid = G > 1 ? p->grain_id : nullptr;
  a.tables = reinterpret_cast<float*>(ws + L.tables);
  // one grain: its rotated table serves every voxel (no per-voxel rotation)
  a.rot = (rotated && G > 1) ? reinterpret_cast<float*>(ws + L.rot) : nullptr;
  if (rotated) {
    // crystal-frame table shared by every grain: [C 21][dC_q 21 x V][eps0_q 6 x V]
    pack_sym(p->C_grain, a.xtab);
    for (int q = 0; q < nv; ++q) {
      double d[36];
      for (int i = 0; i < 36; ++i) d[i] = p->C_var[36 * q + i] - p->C_grain[i];
      pack_sym(d, a.xtab + 21 * (q + 1));
      for (int k = 0; k < 6; ++k) a.xtab[21 * (nv + 1) + 6 * q + k] = (float)p->eps0[6 * q + k];
    }
  }
  a.spec = reinterpret_cast<float2*>(ws + L.spec);
  float2* tw = reinterpret_cast<float2*>(ws + L.tw);
  a.tw_xh = tw;
  a.tw_x = tw + p->nx / 2;
  a.tw_y = tw + p->nx / 2 + p->nx;
  a.tw_z = tw + p->nx / 2 + p->nx + p->ny;
  a.part_ms = reinterpret_cast<double*>(ws + L.part_ms);
  a.part_res = reinterpret_cast<double*>(ws + L.part_res);
  a.part_ac = reinterpret_cast<double*>(ws + L.part_ac);
  a.part_mm = reinterpret_cast<float*>(ws + L.part_mm);
  a.part_gd = reinterpret_cast<double*>(ws + L.part_gd);
  a.state = reinterpret_cast<DevState*>(ws + L.state);
  a.save_stress = 0;

  std::vector<float> twh(2 * (size_t)(p->nx / 2 + p->nx + p->ny + p->nz));
  twiddles(p->nx / 2, twh.data());
  twiddles(p->nx, twh.data() + 2 * (p->nx / 2));
  twiddles(p->ny, twh.data() + 2 * (p->nx / 2 + p->nx));
  twiddles(p->nz, twh.data() + 2 * (p->nx / 2 + p->nx + p->ny));

  DevState st0;
  std::memset(&st0, 0, sizeof(st0));

  hipError_t e;
  if ((e = hipHostMalloc(reinterpret_cast<void**>(&c->host_status), sizeof(Status), hipHostMallocDefault)) !=
      hipSuccess) {
    delete c;
    fprintf(stderr, "pf_init: hipHostMalloc: %s\n", hipGetErrorString(e));
    return PF_EDEVICE;
  }
  std::memset(c->host_status, 0, sizeof(Status));
  auto bail = [&](hipError_t err, const char* what) {
    fprintf(stderr, "pf_init: %s: %s\n", what, hipGetErrorString(err));
    hipHostFree(c->host_status);
    delete c;
    return PF_EDEVICE;
  };
  if ((e = hipMemcpyAsync(const_cast<float*>(a.tables), tab.data(), tab.size() * sizeof(float),
                          hipMemcpyHostToDevice, c->stream)) != hipSuccess)
    return bail(e, "tables");
  if (rotated && (e = hipMemcpyAsync(const_cast<float*>(a.rot), rot.data(), rot.size() * sizeof(float),
                                     hipMemcpyHostToDevice, c->stream)) != hipSuccess)
    return bail(e, "rotations");
  if ((e = hipMemcpyAsync(tw, twh.data(), twh.size() * sizeof(float), hipMemcpyHostToDevice, c->stream)) !=
      hipSuccess)
    return bail(e, "twiddles");
  if ((e = hipMemcpyAsync(a.state, &st0, sizeof(st0), hipMemcpyHostToDevice, c->stream)) != hipSuccess)
    return bail(e, "state");
  if ((e = hipMemcpyAsync(a.eta, p->eta0, sizeof(float) * c->nvox * nv, hipMemcpyDeviceToDevice, c->stream)) !=
      hipSuccess)
    return bail(e, "eta0");
  if ((e = hipMemsetAsync(a.eps, 0, sizeof(float) * c->nvox * 6, c->stream)) != hipSuccess)
    return bail(e, "strain");
  // gradient energy of the initial state
  if ((e = pfl::raw_x_forward(a, a.eta, nv, c->stream)) != hipSuccess) return bail(e, "init x");
  if ((e = pfl::y_pass(a, nv, 1, c->stream)) != hipSuccess) return bail(e, "init y");
  if ((e = pfl::ac_z_update(a, 1, c->stream)) != hipSuccess) return bail(e, "init z");
  if ((e = pfl::ac_finalize(a, 1, c->stream)) != hipSuccess) return bail(e, "init fin");
  if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return bail(e, "init sync");
  *out = c;
  return PF_OK;
}

static int read_status(pf_ctx* c) {
  hipError_t e = hipMemcpyAsync(c->host_status, &c->args.state->st, sizeof(Status), hipMemcpyDeviceToHost,
                                c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "status copy");
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "stream sync");
  return PF_OK;
}

static int ms_iteration(pf_ctx* c, int mode) {
  KArgs a = c->args;
  a.iter_mode = mode;
  hipStream_t s = c->stream;
  PF_TRY(launch(c, "ms_x_forward", [&] { return pfl::ms_x_forward(a, s); }));
  PF_TRY(launch(c, "ms_finalize_mean", [&] { return pfl::ms_finalize_mean(a, s); }));
  PF_TRY(launch(c, "ms_y_forward", [&] { return pfl::y_pass(a, 6, 1, s); }));
  PF_TRY(launch(c, "ms_z_green", [&] { return pfl::ms_z_green(a, s); }));
  PF_TRY(launch(c, "ms_y_inverse", [&] { return pfl::y_pass(a, 6, -1, s); }));
  PF_TRY(launch(c, "ms_x_inverse", [&] { return pfl::ms_x_inverse(a, s); }));
  PF_TRY(launch(c, "ms_finalize_residual", [&] { return pfl::ms_finalize_residual(a, s); }));
  return PF_OK;
}

int pf_step(pf_ctx* c, int32_t n_steps, const pf_load* load) {
  if (!c) return PF_EINVAL;
  if (!load || n_steps < 0) return fail(c, PF_EINVAL, "pf_step: bad arguments");
  if (load->eps_p) c->args.epsp = load->eps_p;
  c->args.save_stress = (load->flags & PF_STEP_SAVE_STRESS) ? 1 : 0;
  const KArgs& a = c->args;
  hipStream_t s = c->stream;
  for (int n = 0; n < n_steps; ++n) {
    // From the third step on, the first iterate extrapolates the strain of
    // the two previous steps; from the second on, the step's starting strain
    // is kept for that.
    const int first_mode = c->one_iteration ? 0 : (c->hist >= 2 ? 2 : (c->hist >= 1 ? 1 : 0));
    KArgs ab = a;
    ab.iter_mode = first_mode;
    PF_TRY(launch(c, "step_begin", [&] { return pfl::step_begin(ab, load->eps_bar, load->sig_bar, s); }));
    if (c->one_iteration) {
      PF_TRY(ms_iteration(c, 0));
    } else {
      bool conv = false;
      for (int k = 0; k < c->ms_max_iter; ++k) {
        PF_TRY(ms_iteration(c, k == 0 ? first_mode : 0));
        PF_TRY(read_status(c));
        if (c->host_status->done) {
          conv = true;
          break;
        }
      }
      if (!conv) {
        char buf[160];
        snprintf(buf, sizeof(buf), "fixed point not converged after %d iterations (residual %.3e)",
                 c->ms_max_iter, c->host_status->residual);
        return fail(c, PF_ENOCONV, buf);
      }
    }
    PF_TRY(launch(c, "ac_x_forward", [&] { return pfl::ac_x_forward(a, s); }));
    PF_TRY(launch(c, "ac_y_forward", [&] { return pfl::y_pass(a, a.nv, 1, s); }));
    PF_TRY(launch(c, "ac_z_update", [&] { return pfl::ac_z_update(a, 0, s); }));
    PF_TRY(launch(c, "ac_y_inverse", [&] { return pfl::y_pass(a, a.nv, -1, s); }));
    PF_TRY(launch(c, "ac_x_inverse", [&] { return pfl::ac_x_inverse(a, s); }));
    PF_TRY(launch(c, "ac_finalize", [&] { return pfl::ac_finalize(a, 0, s); }));
    c->steps += 1;
    c->hist += 1;
  }
  if (n_steps > 0) {
    PF_TRY(read_status(c));
    if (c->host_status->nonfinite) return fail(c, PF_ENONFINITE, "non-finite order parameter");
  }
  return PF_OK;
}

int pf_fields(pf_ctx* c, int32_t which, int32_t set, float* buf) {
  if (!c) return PF_EINVAL;
  if (!buf) return fail(c, PF_EINVAL, "pf_fields: null buffer");
  float* f = nullptr;
  size_t n = 0;
  switch (which) {
    case PF_FIELD_ETA: f = c->args.eta; n = c->nvox * c->nv; break;
    case PF_FIELD_STRAIN: f = c->args.eps; n = c->nvox * 6; break;
    case PF_FIELD_STRESS:
      if (set) return fail(c, PF_EINVAL, "pf_fields: stress is read-only");
      f = c->args.sig; n = c->nvox * 6; break;
    default: return fail(c, PF_EINVAL, "pf_fields: unknown field");
  }
  if (set) c->hist = 0;  // the strain history no longer describes the state
  hipError_t e = set ? hipMemcpyAsync(f, buf, n * sizeof(float), hipMemcpyDeviceToDevice, c->stream)
                     : hipMemcpyAsync(buf, f, n * sizeof(float), hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "pf_fields");
  return PF_OK;
}

int pf_stats_get(pf_ctx* c, pf_stats* out) {
  if (!c || !out) return PF_EINVAL;
  DevState st;
  hipError_t e = hipMemcpyAsync(&st, c->args.state, sizeof(DevState), hipMemcpyDeviceToHost, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "stats copy");
  e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "stats sync");
  const double ntot = (double)c->nvox, dV = c->dx * c->dx * c->dx;
  std::memset(out, 0, sizeof(*out));
  out->step = c->steps;
  out->G_dw = c->args.A * st.stats[0] * dV;
  out->G_me = st.stats[1] * dV;
  for (int k = 0; k < 6; ++k) {
    out->sig_mean[k] = st.stats[2 + k] / ntot;
    out->eps_mean[k] = st.stats[8 + k] / ntot;
  }
  for (int q = 0; q < c->nv; ++q) out->eta_mean[q] = st.stats[14 + q] / ntot;
  out->G_gd = c->kappa * st.stats[pft::kQac] * dV / ntot;
  out->eta_min = st.stats[pft::kQac + 1];
  out->eta_max = st.stats[pft::kQac + 2];
  out->ms_iters = st.st.iters;
  out->ms_residual = st.st.residual;
  if (st.st.nonfinite) return fail(c, PF_ENONFINITE, "non-finite order parameter");
  return PF_OK;
}

int pf_fft(pf_ctx* c, int32_t direction, int32_t ncomp, float* real, void* spec) {
  if (!c) return PF_EINVAL;
  if (!real || !spec || ncomp < 1 || ncomp > 6 || (direction != 1 && direction != -1))
    return fail(c, PF_EINVAL, "pf_fft: bad arguments");
  KArgs a = c->args;
  a.spec = reinterpret_cast<float2*>(spec);
  a.sh = c->nh;  // caller layout: unpadded rows
  hipStream_t s = c->stream;
  if (direction == 1) {
    PF_TRY(launch(c, "fft_x_forward", [&] { return pfl::raw_x_forward(a, real, ncomp, s); }));
    PF_TRY(launch(c, "fft_y_forward", [&] { return pfl::y_pass(a, ncomp, 1, s); }));
    PF_TRY(launch(c, "fft_z_forward", [&] { return pfl::raw_z(a, ncomp, 1, s); }));
  } else {
    PF_TRY(launch(c, "fft_z_inverse", [&] { return pfl::raw_z(a, ncomp, -1, s); }));
    PF_TRY(launch(c, "fft_y_inverse", [&] { return pfl::y_pass(a, ncomp, -1, s); }));
    PF_TRY(launch(c, "fft_x_inverse",
                  [&] { return pfl::raw_x_inverse(a, real, ncomp, (float)(1.0 / (double)c->nvox), s); }));
  }
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
  for (auto& pe : c->prof) {
    hipEventDestroy(pe.start);
    hipEventDestroy(pe.stop);
  }
  for (auto ev : c->ev_pool) hipEventDestroy(ev);
  if (c->host_status) hipHostFree(c->host_status);
  delete c;
  return PF_OK;
}

const char* pf_last_error(const pf_ctx* c) {
  if (!c) return "null context";
  return c->err.c_str();
}

}  // extern "C"
