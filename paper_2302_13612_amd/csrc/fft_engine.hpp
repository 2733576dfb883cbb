// Register/LDS Stockham FFT engine for gfx950.
//
// A pencil of length N is transformed cooperatively by T = N / E threads;
// thread t owns the E elements t + T*m (m = 0..E-1) both before and after
// the transform (the Stockham formulation sorts itself), so global loads and
// stores of a pencil are T-wide contiguous runs. Stages exchange data through
// LDS; each stage of radix R does E/R radix-R butterflies per thread in
// registers. Twiddles come from a float32 table W_N^n = exp(-2 pi i n / N)
// built on the host in double precision and rounded once.
#pragma once
#include <hip/hip_runtime.h>

namespace pft {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }

// Multiply by W_4 = -i (forward, DIR = +1) or +i (inverse, DIR = -1).
template <int DIR>
__device__ __forceinline__ float2 quarter(float2 a) {
  return DIR > 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
}

// Multiply by W_8 = (1 - i)/sqrt2 (forward) or (1 + i)/sqrt2 (inverse).
template <int DIR>
__device__ __forceinline__ float2 eighth(float2 a) {
  constexpr float h = 0.70710678118654752440f;
  return DIR > 0 ? make_float2((a.x + a.y) * h, (a.y - a.x) * h)
                 : make_float2((a.x - a.y) * h, (a.x + a.y) * h);
}

// In-place DFTs of small sizes, natural order in and out:
// X[k] = sum_j v[j] W_R^{jk}, W_R = exp(-DIR * 2 pi i / R).
template <int DIR>
__device__ __forceinline__ void dft2(float2* v) {
  float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <int DIR>
__device__ __forceinline__ void dft3(float2* v) {
  constexpr float s3 = 0.86602540378443864676f;  // sin(pi/3)
  float2 s = cadd(v[1], v[2]);
  float2 d = csub(v[1], v[2]);
  float2 m = make_float2(v[0].x - 0.5f * s.x, v[0].y - 0.5f * s.y);
  float2 r = cscale(quarter<DIR>(d), s3);
  v[0] = cadd(v[0], s);
  v[1] = cadd(m, r);
  v[2] = csub(m, r);
}

template <int DIR>
__device__ __forceinline__ void dft4(float2* v) {
  float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
  float2 t2 = cadd(v[1], v[3]), t3 = quarter<DIR>(csub(v[1], v[3]));
  v[0] = cadd(t0, t2);
  v[2] = csub(t0, t2);
  v[1] = cadd(t1, t3);
  v[3] = csub(t1, t3);
}

// Radix 8 as two radix-4 DFTs (even / odd samples) combined with W_8^k.
template <int DIR>
__device__ __forceinline__ void dft8(float2* v) {
  float2 e[4] = {v[0], v[2], v[4], v[6]};
  float2 o[4] = {v[1], v[3], v[5], v[7]};
  dft4<DIR>(e);
  dft4<DIR>(o);
  o[1] = eighth<DIR>(o[1]);
  o[2] = quarter<DIR>(o[2]);
  o[3] = quarter<DIR>(eighth<DIR>(o[3]));
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = cadd(e[k], o[k]);
    v[k + 4] = csub(e[k], o[k]);
  }
}

template <int R, int DIR>
__device__ __forceinline__ void dft(float2* v) {
  static_assert(R == 2 || R == 3 || R == 4 || R == 8, "unsupported radix");
  if constexpr (R == 2) dft2<DIR>(v);
  else if constexpr (R == 3) dft3<DIR>(v);
  else if constexpr (R == 4) dft4<DIR>(v);
  else dft8<DIR>(v);
}

// --------------------------------------------------- streaming accesses
// Fields and spectra of a pass are touched once per pass and far larger than
// the caches, so the passes that move whole rows or 128-byte column runs
// load and store them with the nontemporal hint (measured at 256^3: the x
// passes 15-27% faster). The Green z pass and the y passes load without the
// hint: the Green pass's 64-byte column runs share lines with the
// neighbouring tile, which the hint evicts.
typedef float f2v_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 gld(const float2* p) {
  const f2v_t v = __builtin_nontemporal_load(reinterpret_cast<const f2v_t*>(p));
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ void gst(float2* p, float2 v) {
  f2v_t w;
  w.x = v.x;
  w.y = v.y;
  __builtin_nontemporal_store(w, reinterpret_cast<f2v_t*>(p));
}

// ----------------------------------------------------------------- plans
template <int... Rs>
struct Radices {};

// E = elements per thread; every radix divides E; product of radices = N.
template <int N> struct Plan;
template <> struct Plan<16>  { static constexpr int E = 4;  using R = Radices<4, 4>; };
template <> struct Plan<24>  { static constexpr int E = 12; using R = Radices<4, 2, 3>; };
template <> struct Plan<32>  { static constexpr int E = 8;  using R = Radices<8, 4>; };
template <> struct Plan<48>  { static constexpr int E = 12; using R = Radices<4, 4, 3>; };
template <> struct Plan<64>  { static constexpr int E = 8;  using R = Radices<8, 8>; };
template <> struct Plan<96>  { static constexpr int E = 12; using R = Radices<4, 4, 2, 3>; };
template <> struct Plan<128> { static constexpr int E = 8;  using R = Radices<8, 4, 4>; };
template <> struct Plan<192> { static constexpr int E = 12; using R = Radices<4, 4, 4, 3>; };
template <> struct Plan<256> { static constexpr int E = 8;  using R = Radices<8, 8, 4>; };
template <> struct Plan<384> { static constexpr int E = 12; using R = Radices<4, 4, 4, 2, 3>; };
template <> struct Plan<512> { static constexpr int E = 8;  using R = Radices<8, 8, 8>; };

// Alternative plans of the y and z passes, picked per grid by the autotuner:
// variant 0 is Plan<N>; variant 1 holds fewer elements per thread (more
// threads per pencil, fewer registers, more exchange stages); variant 2 holds
// more (fewer threads, more registers). Each is the same transform with its
// own radix split, so results differ only by rounding.
template <int N, int K> struct PlanV;
template <int N> struct PlanV<N, 0> { using P = Plan<N>; };
template <> struct PlanV<32, 1>  { struct P { static constexpr int E = 4;  using R = Radices<4, 4, 2>; }; };
template <> struct PlanV<48, 1>  { struct P { static constexpr int E = 6;  using R = Radices<2, 2, 2, 2, 3>; }; };
template <> struct PlanV<64, 1>  { struct P { static constexpr int E = 4;  using R = Radices<4, 4, 4>; }; };
template <> struct PlanV<96, 1>  { struct P { static constexpr int E = 6;  using R = Radices<2, 2, 2, 2, 2, 3>; }; };
template <> struct PlanV<128, 1> { struct P { static constexpr int E = 4;  using R = Radices<4, 4, 4, 2>; }; };
template <> struct PlanV<192, 1> { struct P { static constexpr int E = 6;  using R = Radices<2, 2, 2, 2, 2, 2, 3>; }; };
template <> struct PlanV<256, 1> { struct P { static constexpr int E = 4;  using R = Radices<4, 4, 4, 4>; }; };
template <> struct PlanV<384, 1> { struct P { static constexpr int E = 6;  using R = Radices<2, 2, 2, 2, 2, 2, 2, 3>; }; };
template <> struct PlanV<512, 1> { struct P { static constexpr int E = 4;  using R = Radices<4, 4, 4, 4, 2>; }; };
template <> struct PlanV<32, 2>  { struct P { static constexpr int E = 16; using R = Radices<8, 4>; }; };
template <> struct PlanV<48, 2>  { struct P { static constexpr int E = 24; using R = Radices<4, 4, 3>; }; };
template <> struct PlanV<64, 2>  { struct P { static constexpr int E = 16; using R = Radices<8, 8>; }; };
template <> struct PlanV<96, 2>  { struct P { static constexpr int E = 24; using R = Radices<4, 4, 2, 3>; }; };
template <> struct PlanV<128, 2> { struct P { static constexpr int E = 16; using R = Radices<8, 4, 4>; }; };
template <> struct PlanV<192, 2> { struct P { static constexpr int E = 24; using R = Radices<4, 4, 4, 3>; }; };
template <> struct PlanV<256, 2> { struct P { static constexpr int E = 16; using R = Radices<8, 8, 4>; }; };
template <> struct PlanV<384, 2> { struct P { static constexpr int E = 24; using R = Radices<4, 4, 4, 2, 3>; }; };
template <> struct PlanV<512, 2> { struct P { static constexpr int E = 16; using R = Radices<8, 8, 8>; }; };

// Plans of the x pass (half-length complex transforms of real rows). Fewer
// elements per thread leave registers for the fused per-voxel physics.
template <int M> struct XPlan;
template <> struct XPlan<16>  { static constexpr int E = 4; using R = Radices<4, 4>; };
template <> struct XPlan<24>  { static constexpr int E = 6; using R = Radices<2, 2, 2, 3>; };
template <> struct XPlan<32>  { static constexpr int E = 4; using R = Radices<4, 4, 2>; };
template <> struct XPlan<48>  { static constexpr int E = 6; using R = Radices<2, 2, 2, 2, 3>; };
template <> struct XPlan<64>  { static constexpr int E = 4; using R = Radices<4, 4, 4>; };
template <> struct XPlan<96>  { static constexpr int E = 6; using R = Radices<2, 2, 2, 2, 2, 3>; };
template <> struct XPlan<128> { static constexpr int E = 4; using R = Radices<4, 4, 4, 2>; };
template <> struct XPlan<192> { static constexpr int E = 6; using R = Radices<2, 2, 2, 2, 2, 2, 3>; };
template <> struct XPlan<256> { static constexpr int E = 4; using R = Radices<4, 4, 4, 4>; };

// ------------------------------------------------------------ LDS views
// Orders the LDS accesses of one wavefront's lanes: the compiler moves no
// memory operation across it, and the LDS unit executes a wavefront's
// operations in issue order, so what any lane wrote before it is what every
// lane of the same wavefront reads after it.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One pencil of a row-major tile, padded by one element every 16 to break
// the stride-R bank conflicts of the scatter phases. A row is transformed
// by threads of one wavefront (T divides 64 and rows are contiguous thread
// ranges), so its exchanges need only wavefront order, no block barrier.
struct RowView {
  float2* base;
  __device__ __forceinline__ static int pad(int e) { return e + (e >> 4); }
  __device__ __forceinline__ float2 read(int e) const { return base[pad(e)]; }
  __device__ __forceinline__ void write(int e, float2 v) const { base[pad(e)] = v; }
  __device__ __forceinline__ static void sync() { wave_sync(); }
  __host__ __device__ static constexpr int padded(int n) { return n + (n >> 4); }
};

// One column of a column-interleaved tile: element e of column c at
// base[e * C + c]; the C columns of a wavefront segment are contiguous. A
// column's threads span the block's wavefronts: exchanges need a barrier.
template <int C>
struct ColView {
  float2* base;
  __device__ __forceinline__ float2 read(int e) const { return base[e * C]; }
  __device__ __forceinline__ void write(int e, float2 v) const { base[e * C] = v; }
  __device__ __forceinline__ static void sync() { __syncthreads(); }
};

template <int DIR>
__device__ __forceinline__ float2 twiddle(const float2* __restrict__ tw, int idx) {
  float2 w = tw[idx];
  return DIR > 0 ? w : cconj(w);
}

// Radix list of a plan as constants.
template <class R> struct RadixInfo;
template <int... Rs>
struct RadixInfo<Radices<Rs...>> {
  static constexpr int n = sizeof...(Rs);
  static constexpr int r[n] = {Rs...};
};

// Per-thread twiddles of every stage of plan P in direction DIR. They depend
// only on the thread index, so a thread that transforms several pencils
// loads them once from the table and keeps them in registers (each stage of
// a pencil would otherwise wait on its table loads behind a barrier).
template <int N, class P, int DIR>
struct TwCache {
  using RI = RadixInfo<typename P::R>;
  static constexpr int ns(int s) {
    int v = 1;
    for (int i = 0; i < s; ++i) v *= RI::r[i];
    return v;
  }
  // first twiddle of stage s (stage 0 needs none)
  static constexpr int offset(int s) {
    int v = 0;
    for (int i = 1; i < s; ++i) v += (P::E / RI::r[i]) * (RI::r[i] - 1);
    return v;
  }
  static constexpr int count = offset(RI::n);
  float2 w[count > 0 ? count : 1];

  template <int SI>
  __device__ __forceinline__ void load_stages(const float2* __restrict__ tw, int t) {
    if constexpr (SI < RI::n) {
      constexpr int R = RI::r[SI], NS = ns(SI), NB = P::E / R, T = N / P::E;
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int k = (t + T * q) % NS;
#pragma unroll
        for (int r = 1; r < R; ++r) w[offset(SI) + q * (R - 1) + r - 1] = twiddle<DIR>(tw, r * k * (N / (NS * R)));
      }
      load_stages<SI + 1>(tw, t);
    }
  }
  __device__ __forceinline__ void load(const float2* __restrict__ tw, int t) { load_stages<1>(tw, t); }
  // the same thread's twiddles for the opposite direction (conjugates)
  __device__ __forceinline__ TwCache<N, P, -DIR> conj() const {
    TwCache<N, P, -DIR> c;
#pragma unroll
    for (int i = 0; i < (count > 0 ? count : 1); ++i) c.w[i] = cconj(w[i]);
    return c;
  }
};

// Twiddle r of butterfly q of stage SI (R, NS): from the table, or from a
// thread's cache.
template <int N, class P, int R, int NS, int SI, int DIR>
__device__ __forceinline__ float2 stage_twiddle(const float2* __restrict__ tw, int t, int q, int r) {
  constexpr int T = N / P::E;
  const int k = (t + T * q) % NS;
  return twiddle<DIR>(tw, r * k * (N / (NS * R)));
}
template <int N, class P, int R, int NS, int SI, int DIR>
__device__ __forceinline__ float2 stage_twiddle(const TwCache<N, P, DIR>& c, int, int q, int r) {
  return c.w[TwCache<N, P, DIR>::offset(SI) + q * (R - 1) + r - 1];
}

// One Stockham stage. NS = product of the radices of earlier stages, SI =
// stage index. FIRST: inputs from registers; LAST: outputs to registers.
// Every LDS write phase sits between two syncs of the view, so callers may
// reuse the buffer. TW: the twiddle table (const float2*) or a TwCache.
template <int N, class P, int R, int NS, int SI, int DIR, bool FIRST, bool LAST, class View, class TW>
__device__ __forceinline__ void stockham_stage(float2 (&v)[P::E], const View& lds, int t, const TW& tw) {
  constexpr int E = P::E;
  constexpr int T = N / E;
  constexpr int NB = E / R;  // butterflies per thread
  static_assert(E % R == 0, "radix must divide elements per thread");
  float2 a[E];
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int j = t + T * q;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if constexpr (FIRST) a[q * R + r] = v[q + r * NB];
      else a[q * R + r] = lds.read(j + r * (N / R));
    }
    if constexpr (!FIRST) {
#pragma unroll
      for (int r = 1; r < R; ++r)
        a[q * R + r] = cmul(a[q * R + r], stage_twiddle<N, P, R, NS, SI, DIR>(tw, t, q, r));
    }
    dft<R, DIR>(&a[q * R]);
  }
  if constexpr (LAST) {
#pragma unroll
    for (int q = 0; q < NB; ++q)
#pragma unroll
      for (int r = 0; r < R; ++r) v[q + r * NB] = a[q * R + r];
  } else {
    View::sync();
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int j = t + T * q;
      const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
      for (int r = 0; r < R; ++r) lds.write(base + r * NS, a[q * R + r]);
    }
    View::sync();
  }
}

template <int N, class P, int NS, int SI, int DIR, bool FIRST, class View, class TW, int R0, int... Rest>
__device__ __forceinline__ void run_stages(float2 (&v)[P::E], const View& lds, int t, const TW& tw,
                                           Radices<R0, Rest...>) {
  constexpr bool LAST = sizeof...(Rest) == 0;
  stockham_stage<N, P, R0, NS, SI, DIR, FIRST, LAST>(v, lds, t, tw);
  if constexpr (!LAST) run_stages<N, P, NS * R0, SI + 1, DIR, false>(v, lds, t, tw, Radices<Rest...>{});
}

// Transform the pencil held in v (thread t owns elements t + T*m, T = N/E)
// in place with plan P. All threads that share the view's sync (the
// wavefront of a row, the block of a column tile) must call it together. tw: the twiddle table or the thread's TwCache.
template <int N, int DIR, class P = Plan<N>, class View, class TW>
__device__ __forceinline__ void fft_pencil(float2 (&v)[P::E], const View& lds, int t, const TW& tw) {
  run_stages<N, P, 1, 0, DIR, true>(v, lds, t, tw, typename P::R{});
}

// NC pencils of one block transformed in lockstep: every stage's LDS
// exchange of all NC pencils (disjoint views) shares one pair of barriers.
template <int N, class P, int R, int NS, int SI, int DIR, bool FIRST, bool LAST, int NC, class View, class TW>
__device__ __forceinline__ void stockham_stage_n(float2 (&v)[NC][P::E], const View (&lds)[NC], int t, const TW& tw) {
  constexpr int E = P::E;
  constexpr int T = N / E;
  constexpr int NB = E / R;
  static_assert(E % R == 0, "radix must divide elements per thread");
  float2 a[NC][E];
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int j = t + T * q;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if constexpr (FIRST) a[c][q * R + r] = v[c][q + r * NB];
        else a[c][q * R + r] = lds[c].read(j + r * (N / R));
      }
      if constexpr (!FIRST) {
#pragma unroll
        for (int r = 1; r < R; ++r)
          a[c][q * R + r] = cmul(a[c][q * R + r], stage_twiddle<N, P, R, NS, SI, DIR>(tw, t, q, r));
      }
      dft<R, DIR>(&a[c][q * R]);
    }
  if constexpr (LAST) {
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int q = 0; q < NB; ++q)
#pragma unroll
        for (int r = 0; r < R; ++r) v[c][q + r * NB] = a[c][q * R + r];
  } else {
    View::sync();
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        const int j = t + T * q;
        const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
        for (int r = 0; r < R; ++r) lds[c].write(base + r * NS, a[c][q * R + r]);
      }
    View::sync();
  }
}

template <int N, class P, int NS, int SI, int DIR, bool FIRST, int NC, class View, class TW, int R0, int... Rest>
__device__ __forceinline__ void run_stages_n(float2 (&v)[NC][P::E], const View (&lds)[NC], int t, const TW& tw,
                                             Radices<R0, Rest...>) {
  constexpr bool LAST = sizeof...(Rest) == 0;
  stockham_stage_n<N, P, R0, NS, SI, DIR, FIRST, LAST, NC>(v, lds, t, tw);
  if constexpr (!LAST) run_stages_n<N, P, NS * R0, SI + 1, DIR, false, NC>(v, lds, t, tw, Radices<Rest...>{});
}

template <int N, int DIR, class P, int NC, class View, class TW>
__device__ __forceinline__ void fft_pencils(float2 (&v)[NC][P::E], const View (&lds)[NC], int t, const TW& tw) {
  run_stages_n<N, P, 1, 0, DIR, true, NC>(v, lds, t, tw, typename P::R{});
}

}  // namespace pft
