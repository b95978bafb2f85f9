// Batched Newton-Raphson power flow for meshed grids (Sec. II-A), one
// workgroup per scenario, and its adjoint.
//
// A workgroup owns one scenario for its whole solve: every vector of length n
// (buses) or m = |Theta| + |Q| (Newton state) is split over the workgroup's
// threads by rows (thread t owns rows t, t + BLOCK, ...), so per-scenario dot
// products and norms are workgroup reductions and no grid-wide
// synchronisation is ever needed.  Per-scenario data:
//   * LDS (about 39 KB at 2000 buses in FP64, so four workgroups share a CU):
//     the vector being gathered (V for Ybus V, the direction of the
//     Jacobian-vector product, the preconditioner's work vector), the packed
//     Hessenberg matrix and the Givens rotations;
//   * registers: the current Krylov vector w;
//   * HBM (scenario-major workspace): theta, |V|, 1/|V|, V, I, F, the Newton step
//     and the Krylov basis, always accessed at the thread's own rows, so
//     consecutive lanes touch consecutive addresses.
// The shared network data (Ybus, factors of B' and B'') is read through the
// caches by every workgroup; its descriptor sits in device memory.
//
// Steps per Newton iteration (eqs. (1)-(3), (7)-(9)):
//   mismatch  V = |V| e^{j theta}, I = Ybus V, S = V conj(I),
//             F = [Re S - P on Theta ; Im S - Q on Q], max |F|
//   GMRES     left-preconditioned restarted GMRES on J dx = -F with
//             Jacobian-vector products dS = dV conj(I) + V conj(Ybus dV),
//             dV = V (j dtheta + d|V| / |V|), the preconditioner applied by
//             forward block substitution, classical Gram-Schmidt with a second
//             pass whenever the first cancels more than 1 - 1/sqrt(2) of the
//             norm (Kahan-Parlett), Givens rotations on the Hessenberg matrix
//   update    theta += dx_theta, |V| += dx_|V|   (FP64)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "tx.hpp"

namespace pfx {

namespace {

constexpr int WAVE = 64;

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

// max that propagates NaN
__device__ __forceinline__ double nanmax(double a, double b) {
  if (a != a) return a;
  if (b != b) return b;
  return a > b ? a : b;
}

__device__ __forceinline__ double wave_nanmax(double v) {
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) v = nanmax(v, __shfl_xor(v, off, WAVE));
  return v;
}

// Workgroup sum; every thread gets the same result.  Ends with a barrier so
// `red` can be reused right away.
template <typename T, int BLOCK>
__device__ T block_sum(T v, T* red) {
  constexpr int NW = BLOCK / WAVE;
  v = wave_sum(v);
  if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = v;
  __syncthreads();
  T s = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) s += red[i];
  __syncthreads();
  return s;
}

template <int BLOCK>
__device__ double block_nanmax(double v, double* red) {
  constexpr int NW = BLOCK / WAVE;
  v = wave_nanmax(v);
  if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = v;
  __syncthreads();
  double s = red[0];
#pragma unroll
  for (int i = 1; i < NW; ++i) s = nanmax(s, red[i]);
  __syncthreads();
  return s;
}

// Runtime-indexed access to a register array through a select chain, so that
// loops with heavy bodies can stay rolled while the array stays in registers.
template <typename T, int K>
__device__ __forceinline__ T rget(const T (&w)[K], int k) {
  T v = w[0];
#pragma unroll
  for (int q = 1; q < K; ++q)
    if (q == k) v = w[q];
  return v;
}

template <typename T, int K>
__device__ __forceinline__ void rset(T (&w)[K], int k, T v) {
#pragma unroll
  for (int q = 0; q < K; ++q)
    if (q == k) w[q] = v;
}

// Row k of thread t is t + k BLOCK.  Per-scenario state vectors are padded to
// kd BLOCK rows (zeros past m), so the streaming loops carry no row guards.
template <int BLOCK>
__device__ __forceinline__ unsigned row(int k) {
  return threadIdx.x + (unsigned)k * BLOCK;
}

// Global-memory element access by a 32-bit index from a base pointer that is
// uniform across the workgroup: the byte offset stays 32-bit and the pointer
// is tagged global, so the scalar-base plus vector-offset form is used instead
// of a 64-bit address per element.
template <typename T>
__device__ __forceinline__ T gld(const T* base, unsigned i) {
  typedef __attribute__((address_space(1))) const char GC;
  typedef __attribute__((address_space(1))) const T GT;
  return *(GT*)((GC*)base + i * (unsigned)sizeof(T));
}

template <typename T>
__device__ __forceinline__ void gst(T* base, unsigned i, T v) {
  typedef __attribute__((address_space(1))) char GC;
  typedef __attribute__((address_space(1))) T GT;
  *(GT*)((GC*)base + i * (unsigned)sizeof(T)) = v;
}

struct NrLayout {
  int xs, tmp, red, h1, h2, H, cs, sn, g, y, misc, total;
};

__host__ __device__ inline int align16(int x) { return (x + 15) & ~15; }

// Column j of the packed Hessenberg matrix holds rows 0..j+1 at offset j(j+3)/2.
__host__ __device__ inline int hcol(int j) { return j * (j + 3) / 2; }

__host__ __device__ inline NrLayout nr_layout(int n, int m, int kmax, int R, int NW, int ts) {
  NrLayout L;
  int o = 0;
  const int xs_bytes = m * ts > 2 * n * 8 ? m * ts : 2 * n * 8;
  L.xs = o;   o += align16(xs_bytes);
  L.tmp = o;  o += align16((kmax > 0 ? kmax : 1) * ts);
  const int red_bytes = (R + 2) * NW * ts > NW * 8 ? (R + 2) * NW * ts : NW * 8;
  L.red = o;  o += align16(red_bytes);
  L.h1 = o;   o += align16((R + 2) * ts);
  L.h2 = o;   o += align16((R + 2) * ts);
  L.H = o;    o += align16(hcol(R) * ts);
  L.cs = o;   o += align16(R * ts);
  L.sn = o;   o += align16(R * ts);
  L.g = o;    o += align16((R + 1) * ts);
  L.y = o;    o += align16(R * ts);
  L.misc = o; o += 64;
  L.total = o;
  return L;
}

template <typename T>
struct Smem {
  T* xs;
  double* vs;
  T* tmp;
  T* red;
  double* redd;
  T* h1;
  T* h2;
  T* H;
  T* cs;
  T* sn;
  T* g;
  T* yv;
  T* misc;
};

template <typename T>
__device__ Smem<T> carve(unsigned char* smem, const NrLayout& L) {
  Smem<T> s;
  s.xs = reinterpret_cast<T*>(smem + L.xs);
  s.vs = reinterpret_cast<double*>(smem + L.xs);
  s.tmp = reinterpret_cast<T*>(smem + L.tmp);
  s.red = reinterpret_cast<T*>(smem + L.red);
  s.redd = reinterpret_cast<double*>(smem + L.red);
  s.h1 = reinterpret_cast<T*>(smem + L.h1);
  s.h2 = reinterpret_cast<T*>(smem + L.h2);
  s.H = reinterpret_cast<T*>(smem + L.H);
  s.cs = reinterpret_cast<T*>(smem + L.cs);
  s.sn = reinterpret_cast<T*>(smem + L.sn);
  s.g = reinterpret_cast<T*>(smem + L.g);
  s.yv = reinterpret_cast<T*>(smem + L.y);
  s.misc = reinterpret_cast<T*>(smem + L.misc);
  return s;
}

// ---------------------------------------------------------------------------
// Solve (B + eps I) x = b in place for the vector held in LDS in factor order
// (see factor.hpp).  The factor is A = L D L^T with unit lower L over the
// sparse prefix and the explicit inverse of the Schur complement S over the
// dense core:
//   y1 = L11^-1 b1 (levels), t = b2 - L21 y1, x2 = S^-1 t, w1 = D11^-1 y1,
//   x1 = L11^-T (w1 - L21^T x2) (levels, reverse order).
// Ends with a barrier.
template <typename T, int BLOCK>
__device__ void spd_apply(const SpdDev<T>& f, T* xs, T* tmp) {
  for (int l = 0; l < f.nfl; ++l) {
    const int s = gld(f.f_lev, l), e = gld(f.f_lev, l + 1);
    for (int q = s + (int)threadIdx.x; q < e; q += BLOCK) {
      const int i = gld(f.f_rows, q);
      T a = xs[i];
      const int pe = gld(f.L_ptr, i + 1);
      for (int p = gld(f.L_ptr, i); p < pe; ++p) a -= gld(f.L_val, p) * xs[gld(f.L_col, p)];
      xs[i] = a;
    }
    __syncthreads();
  }
  if (f.k > 0) {
    for (int i = f.c + (int)threadIdx.x; i < f.N; i += BLOCK) {
      T a = xs[i];
      const int pe = gld(f.L_ptr, i + 1);
      for (int p = gld(f.L_ptr, i); p < pe; ++p) a -= gld(f.L_val, p) * xs[gld(f.L_col, p)];
      tmp[i - f.c] = a;
    }
    __syncthreads();
    for (int i = (int)threadIdx.x; i < f.k; i += BLOCK) {
      T a0 = 0, a1 = 0;
      unsigned o = i;
      int l = 0;
      for (; l + 1 < f.k; l += 2, o += 2 * f.k) {
        a0 += gld(f.Sinv, o) * tmp[l];
        a1 += gld(f.Sinv, o + f.k) * tmp[l + 1];
      }
      if (l < f.k) a0 += gld(f.Sinv, o) * tmp[l];
      xs[f.c + i] = a0 + a1;
    }
  }
  for (int j = (int)threadIdx.x; j < f.c; j += BLOCK) xs[j] *= gld(f.dinv, j);
  __syncthreads();
  for (int l = 0; l < f.nbl; ++l) {
    const int s = gld(f.b_lev, l), e = gld(f.b_lev, l + 1);
    for (int q = s + (int)threadIdx.x; q < e; q += BLOCK) {
      const int j = gld(f.b_rows, q);
      T a = xs[j];
      const int pe = gld(f.T_ptr, j + 1);
      for (int p = gld(f.T_ptr, j); p < pe; ++p) a -= gld(f.T_val, p) * xs[gld(f.T_col, p)];
      xs[j] = a;
    }
    __syncthreads();
  }
}

// Per-scenario views into the FP64 workspace (7 n + 2 mp doubles, mp = kd
// BLOCK >= m the padded state length).
struct Scen {
  double* th;   // [n] angle
  double* vm;   // [n] magnitude
  double* ivm;  // [n] 1 / magnitude
  double* vre;  // [n] V
  double* vim;
  double* ire;  // [n] I = Ybus V
  double* iim;
  double* F;    // [mp] mismatch, then the GMRES right-hand side (zero past m)
  double* dx;   // [mp] Newton step
};

__device__ inline Scen scen_at(double* ws, int n, unsigned mp) {
  return Scen{ws, ws + n, ws + 2 * n, ws + 3 * n, ws + 4 * n, ws + 5 * n, ws + 6 * n, ws + 7 * n,
              ws + 7 * n + mp};
}

// z = M^-1 w for the left preconditioner of eq. (7), by the forward block
// substitution of eqs. (8)-(9):
//   z_Theta = (B' + eps I)^-1 diag(|V_Theta|)^-1 w_Theta
//   z_Q     = (B'' + eps I)^-1 diag(|V_Q|)^-1 (w_Q - G z_Theta)
template <typename T, int BLOCK, int K>
__device__ void precond(const TxDev<T>& net, const Scen& sc, int kd, T (&w)[K], T* xs, T* tmp) {
  const unsigned nth = net.nth, m = net.m;
  T* x1 = xs;
  T* x2 = xs + nth;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const unsigned r = row<BLOCK>(k);
    if (k < kd && r < nth) x1[gld(net.bp.pinv, r)] = w[k] * (T)gld(sc.ivm, r);
  }
  __syncthreads();
  spd_apply<T, BLOCK>(net.bp, x1, tmp);
  if (net.npq > 0) {
#pragma unroll 1
    for (int k = 0; k < kd; ++k) {
      const unsigned r = row<BLOCK>(k);
      if (r >= nth && r < m) {
        const unsigned q = r - nth;
        T t = rget(w, k);
        const int pe = gld(net.g_ptr, q + 1);
        for (int p = gld(net.g_ptr, q); p < pe; ++p) t -= gld(net.g_val, p) * x1[gld(net.g_col, p)];
        x2[gld(net.bpp.pinv, q)] = t * (T)gld(sc.ivm, q);
      }
    }
    __syncthreads();
    spd_apply<T, BLOCK>(net.bpp, x2, tmp);
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const unsigned r = row<BLOCK>(k);
    if (k < kd) {
      if (r < nth) w[k] = x1[gld(net.bp.pinv, r)];
      else if (r < m) w[k] = x2[gld(net.bpp.pinv, r - nth)];
    }
  }
  __syncthreads();
}

// w <- J w, the Jacobian of the mismatch at the current V (with I = Ybus V).
template <typename T, int BLOCK, int K>
__device__ void jvp(const TxDev<T>& net, const Scen& sc, int kd, T (&w)[K], T* xs) {
  const int nth = net.nth, npq = net.npq;
  const unsigned m = net.m;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const unsigned r = row<BLOCK>(k);
    if (k < kd && r < m) xs[r] = w[k];
  }
  __syncthreads();
  // dV_b = V_b (j p_theta + p_|V| / |V|)
  auto dv = [&](int bus, T& dr, T& di) {
    const T pth = bus < nth ? xs[bus] : (T)0;
    const T a = bus < npq ? xs[nth + bus] * (T)gld(sc.ivm, bus) : (T)0;
    const T vr = (T)gld(sc.vre, bus), vi = (T)gld(sc.vim, bus);
    dr = vr * a - vi * pth;
    di = vi * a + vr * pth;
  };
#pragma unroll 1
  for (int k = 0; k < kd; ++k) {
    const unsigned r = row<BLOCK>(k);
    if (r < m) {
      const int i = (int)r < nth ? (int)r : (int)r - nth;
      T dIr = 0, dIi = 0;
      const int pe = gld(net.y_ptr, i + 1);
      for (int p = gld(net.y_ptr, i); p < pe; ++p) {
        T dr, di;
        dv(gld(net.y_col, p), dr, di);
        const T yr = (T)gld(net.y_re, p), yi = (T)gld(net.y_im, p);
        dIr += yr * dr - yi * di;
        dIi += yr * di + yi * dr;
      }
      T dVr, dVi;
      dv(i, dVr, dVi);
      const T Ir = (T)gld(sc.ire, i), Ii = (T)gld(sc.iim, i);
      const T vr = (T)gld(sc.vre, i), vi = (T)gld(sc.vim, i);
      // dS = dV conj(I) + V conj(dI): real part on Theta rows, imaginary on Q rows
      rset(w, k, (int)r < nth ? dVr * Ir + dVi * Ii + vr * dIr + vi * dIi
                              : dVi * Ir - dVr * Ii + vi * dIr - vr * dIi);
    }
  }
  __syncthreads();
}

// h[i] = <basis_i, w> for i < nv and, if `ss` is not null, h[nv] = sum of *ss
// over the workgroup.  Results in LDS h; ends with a barrier.
template <typename T, int BLOCK, int K>
__device__ void multi_dot(const T* basis, unsigned stride, int nv, int kd, const T (&w)[K], const T* ss,
                          T* red, T* h) {
  constexpr int NW = BLOCK / WAVE;
  const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
  int i = 0;
  for (; i + 1 < nv; i += 2) {
    const T* v0 = basis + (unsigned)i * stride;
    const T* v1 = v0 + stride;
    T a0 = 0, a1 = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (k < kd) {
        a0 += gld(v0, row<BLOCK>(k)) * w[k];
        a1 += gld(v1, row<BLOCK>(k)) * w[k];
      }
    }
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    if (lane == 0) {
      red[i * NW + wid] = a0;
      red[(i + 1) * NW + wid] = a1;
    }
  }
  if (i < nv) {
    const T* v0 = basis + (unsigned)i * stride;
    T a0 = 0;
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (k < kd) a0 += gld(v0, row<BLOCK>(k)) * w[k];
    a0 = wave_sum(a0);
    if (lane == 0) red[i * NW + wid] = a0;
  }
  const int nout = ss ? nv + 1 : nv;
  if (ss) {
    const T a = wave_sum(*ss);
    if (lane == 0) red[nv * NW + wid] = a;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < nout; q += BLOCK) {
    T s = 0;
#pragma unroll
    for (int u = 0; u < NW; ++u) s += red[q * NW + u];
    h[q] = s;
  }
  __syncthreads();
}

// w -= sum_i h[i] basis_i
template <typename T, int BLOCK, int K>
__device__ void subtract_proj(const T* basis, unsigned stride, int nv, int kd, T (&w)[K], const T* h) {
  int i = 0;
  for (; i + 1 < nv; i += 2) {
    const T h0 = h[i], h1 = h[i + 1];
    const T* v0 = basis + (unsigned)i * stride;
    const T* v1 = v0 + stride;
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (k < kd) w[k] -= h0 * gld(v0, row<BLOCK>(k)) + h1 * gld(v1, row<BLOCK>(k));
  }
  if (i < nv) {
    const T h0 = h[i];
    const T* v0 = basis + (unsigned)i * stride;
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (k < kd) w[k] -= h0 * gld(v0, row<BLOCK>(k));
  }
}

// Mismatch at the current (theta, |V|): writes V, 1/|V|, I and F to the
// workspace and returns max |F| (NaN if any entry is NaN).
template <typename T, int BLOCK, int K>
__device__ double mismatch(const TxDev<T>& net, const Scen& sc, int kd, const double* P, const double* Q,
                           double* vs, double* red) {
  const int n = net.n, nth = net.nth, m = net.m;
  const int* ext = net.int2ext;
  for (int i = threadIdx.x; i < n; i += BLOCK) {
    double s, c;
    sincos(gld(sc.th, i), &s, &c);
    const double vm = gld(sc.vm, i);
    const double vr = vm * c, vi = vm * s;
    gst(sc.vre, i, vr);
    gst(sc.vim, i, vi);
    gst(sc.ivm, i, 1.0 / vm);
    vs[2 * i] = vr;
    vs[2 * i + 1] = vi;
  }
  __syncthreads();
  double fmax = 0.0;
#pragma unroll 1
  for (int k = 0; k < kd; ++k) {
    const int r = (int)row<BLOCK>(k);
    if (r >= m) {
      gst(sc.F, r, 0.0);  // padding rows of the right-hand side stay zero
    } else {
      const int i = r < nth ? r : r - nth;
      double Ir = 0.0, Ii = 0.0;
      const int pe = gld(net.y_ptr, i + 1);
      for (int p = gld(net.y_ptr, i); p < pe; ++p) {
        const int c = gld(net.y_col, p);
        const double yr = gld(net.y_re, p), yi = gld(net.y_im, p);
        const double vr = vs[2 * c], vi = vs[2 * c + 1];
        Ir += yr * vr - yi * vi;
        Ii += yr * vi + yi * vr;
      }
      const double vr = vs[2 * i], vi = vs[2 * i + 1];
      double f;
      if (r < nth) {
        gst(sc.ire, i, Ir);
        gst(sc.iim, i, Ii);
        f = vr * Ir + vi * Ii - gld(P, gld(ext, i));
      } else {
        f = vi * Ir - vr * Ii - gld(Q, gld(ext, i));
      }
      gst(sc.F, r, f);
      fmax = nanmax(fmax, fabs(f));
    }
  }
  return block_nanmax<BLOCK>(fmax, red);
}

// Algorithmic HBM bytes of one scenario (the byte model reported with the
// solve): with w = sizeof(T), per Jacobian-vector product 2 w m + 32 n, per
// preconditioner application 2 w m + 8 n, per Gram-Schmidt pass of Arnoldi
// step j (against j + 1 vectors) (2 j + 3) w m, per cycle start 8 m + w m,
// per cycle end (k + 2) w m, per mismatch evaluation 32 n + 16 m and per
// Newton update 16 m.
struct ByteModel {
  double wm, m8, n8;
  __device__ double jvp() const { return 2 * wm + 4 * n8; }
  __device__ double pre() const { return 2 * wm + n8; }
  __device__ double orth_pass(int j) const { return (2.0 * j + 3.0) * wm; }
  __device__ double mismatch() const { return 4 * n8 + 2 * m8; }
  __device__ double update() const { return 2 * m8; }
};

// Restarted GMRES with left preconditioning for A x = b from x = 0, where
// apply_a(w) overwrites w with A w and apply_m(w) with M^-1 w (both on the
// thread's own rows).  b is read from `rhs` (FP64, own rows); x accumulates in
// FP64 in `x` (own rows).  Stops when the Givens estimate of
// ||M^-1 (b - A x)|| reaches rtol ||M^-1 b||, after max_restarts cycles, or at
// a breakdown.  Returns the number of Arnoldi steps; *converged tells whether
// the tolerance was met.
template <typename T, int BLOCK, int K, typename ApplyA, typename ApplyM>
__device__ int gmres_solve(ApplyA&& apply_a, ApplyM&& apply_m, const double* rhs, double* x, T* basis,
                           unsigned mp, int kd, int R, int max_restarts, T rtol, const Smem<T>& s,
                           bool* converged, const ByteModel& bm, double* work) {
  T w[K];
  T beta0 = 0;
  int total = 0;
  bool done = false;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    w[k] = 0;
    if (k < kd) gst(x, row<BLOCK>(k), 0.0);
  }
  for (int cycle = 0; cycle < max_restarts && !done; ++cycle) {
    *work += (cycle > 0 ? bm.jvp() : 0.0) + bm.pre() + bm.m8 + bm.wm;
    if (cycle == 0) {
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (k < kd) w[k] = (T)gld(rhs, row<BLOCK>(k));
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (k < kd) w[k] = (T)gld(x, row<BLOCK>(k));
      apply_a(w);
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (k < kd) w[k] = (T)gld(rhs, row<BLOCK>(k)) - w[k];
    }
    apply_m(w);
    T ss = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) ss += w[k] * w[k];
    const T beta = sqrt(block_sum<T, BLOCK>(ss, s.red));
    if (cycle == 0) beta0 = beta;
    if (!(beta > rtol * beta0) || beta == (T)0) {
      done = !(beta > rtol * beta0);
      break;
    }
    const T ib = (T)1 / beta;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      w[k] *= ib;
      if (k < kd) gst(basis, row<BLOCK>(k), w[k]);
    }
    if (threadIdx.x == 0) s.g[0] = beta;
    int steps = 0;
    T res = beta;
    for (int j = 0; j < R; ++j) {
      apply_a(w);
      apply_m(w);
      T ss0 = 0;
#pragma unroll
      for (int k = 0; k < K; ++k) ss0 += w[k] * w[k];
      multi_dot<T, BLOCK, K>(basis, mp, j + 1, kd, w, &ss0, s.red, s.h1);
      subtract_proj<T, BLOCK, K>(basis, mp, j + 1, kd, w, s.h1);
      T s1 = 0;
#pragma unroll
      for (int k = 0; k < K; ++k) s1 += w[k] * w[k];
      T nrm2 = block_sum<T, BLOCK>(s1, s.red);
      // second pass when the first removed more than 1 - 1/sqrt(2) of the norm
      const bool again = nrm2 < (T)0.5 * s.h1[j + 1];
      if (again) {
        multi_dot<T, BLOCK, K>(basis, mp, j + 1, kd, w, nullptr, s.red, s.h2);
        subtract_proj<T, BLOCK, K>(basis, mp, j + 1, kd, w, s.h2);
        T s2 = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) s2 += w[k] * w[k];
        nrm2 = block_sum<T, BLOCK>(s2, s.red);
      }
      *work += bm.jvp() + bm.pre() + (again ? 2 : 1) * bm.orth_pass(j);
      const T hn = sqrt(nrm2);
      if (threadIdx.x == 0) {
        T* Hj = s.H + hcol(j);
        for (int i = 0; i <= j; ++i) Hj[i] = again ? s.h1[i] + s.h2[i] : s.h1[i];
        Hj[j + 1] = hn;
        for (int i = 0; i < j; ++i) {
          const T t = s.cs[i] * Hj[i] + s.sn[i] * Hj[i + 1];
          Hj[i + 1] = -s.sn[i] * Hj[i] + s.cs[i] * Hj[i + 1];
          Hj[i] = t;
        }
        const T d = sqrt(Hj[j] * Hj[j] + Hj[j + 1] * Hj[j + 1]);
        const T c = d == (T)0 ? (T)1 : Hj[j] / d;
        const T sn = d == (T)0 ? (T)0 : Hj[j + 1] / d;
        s.cs[j] = c;
        s.sn[j] = sn;
        Hj[j] = d;
        Hj[j + 1] = 0;
        s.g[j + 1] = -sn * s.g[j];
        s.g[j] = c * s.g[j];
        s.misc[0] = fabs(s.g[j + 1]);
      }
      __syncthreads();
      res = s.misc[0];
      steps = j + 1;
      if (!(res > rtol * beta0) || j == R - 1 || !(hn > (T)0)) break;
      const T ih = (T)1 / hn;
      T* vnext = basis + (unsigned)(j + 1) * mp;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        w[k] *= ih;
        if (k < kd) gst(vnext, row<BLOCK>(k), w[k]);
      }
    }
    total += steps;
    *work += (steps + 2) * bm.wm;
    // y = H^-1 g (upper triangular after the rotations)
    if (threadIdx.x == 0) {
      for (int i = steps - 1; i >= 0; --i) {
        T a = s.g[i];
        for (int l = i + 1; l < steps; ++l) a -= s.H[hcol(l) + i] * s.yv[l];
        const T d = s.H[hcol(i) + i];
        s.yv[i] = d != (T)0 ? a / d : (T)0;
      }
    }
    __syncthreads();
#pragma unroll 1
    for (int k = 0; k < kd; ++k) {
      const unsigned r = row<BLOCK>(k);
      double acc = gld(x, r);
      for (int i = 0; i < steps; ++i) acc += (double)s.yv[i] * (double)gld(basis, (unsigned)i * mp + r);
      gst(x, r, acc);
    }
    done = !(res > rtol * beta0);
    __syncthreads();
  }
  *converged = done;
  return total;
}

template <typename T, int BLOCK, int K>
// Four waves per SIMD: with about 39 KB of LDS per scenario, four workgroups
// (four scenarios) share a CU; registers are capped to match.
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void nr_kernel(const TxDev<T>* __restrict__ netp, NRLaunch a) {
  constexpr int NW = BLOCK / WAVE;
  extern __shared__ __align__(16) unsigned char smem[];
  const TxDev<T>& net = *netp;
  const int b = blockIdx.x;
  const int n = net.n, nth = net.nth, npq = net.npq, m = net.m;
  const int R = a.restart;
  const int kmax = net.bp.k > net.bpp.k ? net.bp.k : net.bpp.k;
  const NrLayout L = nr_layout(n, m, kmax, R, NW, (int)sizeof(T));
  const Smem<T> s = carve<T>(smem, L);
  const int kd = ((n > m ? n : m) + BLOCK - 1) / BLOCK;
  const unsigned mp = (unsigned)kd * BLOCK;

  const Scen sc = scen_at(a.ws_d + (int64_t)b * a.ws_d_stride, n, mp);
  T* basis = reinterpret_cast<T*>(a.ws_basis) + (int64_t)b * a.ws_b_stride;
  const double* P = a.p_inj + (int64_t)b * a.ld;
  const double* Q = a.q_inj + (int64_t)b * a.ld;
  const double* VS = a.vm_set + (int64_t)b * a.ld;
  const int* ext = net.int2ext;

  // flat start: theta = 0, |V| = set-point at PV and slack, 1 at PQ buses
  for (int i = threadIdx.x; i < n; i += BLOCK) {
    gst(sc.th, i, 0.0);
    gst(sc.vm, i, i < npq ? 1.0 : gld(VS, gld(ext, i)));
  }
  __syncthreads();

  auto apply_j = [&](T (&w)[K]) { jvp<T, BLOCK, K>(net, sc, kd, w, s.xs); };
  auto apply_m = [&](T (&w)[K]) { precond<T, BLOCK, K>(net, sc, kd, w, s.xs, s.tmp); };

  int newton = 0, gtotal = 0;
  bool conv = false;
  double fnorm = 0.0;
  const ByteModel bm{(double)sizeof(T) * m, 8.0 * m, 8.0 * n};
  double work = 0.0;
  for (;;) {
    work += bm.mismatch();
    fnorm = mismatch<T, BLOCK, K>(net, sc, kd, P, Q, s.vs, s.redd);
    if (!(fnorm <= a.diverge)) break;
    if (fnorm <= a.tol) {
      conv = true;
      break;
    }
    if (newton >= a.max_newton) break;
    // right-hand side -F in place (own rows)
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (k < kd) gst(sc.F, row<BLOCK>(k), -gld(sc.F, row<BLOCK>(k)));
    bool lin_ok;
    gtotal += gmres_solve<T, BLOCK, K>(apply_j, apply_m, sc.F, sc.dx, basis, mp, kd, R, a.max_restarts,
                                       (T)a.rtol, s, &lin_ok, bm, &work);
    // Newton update (eq. (3)), FP64, own rows
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int r = (int)row<BLOCK>(k);
      if (k < kd) {
        if (r < nth) gst(sc.th, r, gld(sc.th, r) + gld(sc.dx, r));
        else if (r < m) gst(sc.vm, r - nth, gld(sc.vm, r - nth) + gld(sc.dx, r));
      }
    }
    work += bm.update();
    __syncthreads();
    ++newton;
  }

  double* vout = a.v_out + 2 * (int64_t)b * a.ld;
  for (int i = threadIdx.x; i < n; i += BLOCK) {
    const int e = gld(ext, i);
    gst(vout, 2 * e, gld(sc.vre, i));
    gst(vout, 2 * e + 1, gld(sc.vim, i));
  }
  if (threadIdx.x == 0) {
    a.newton_iters[b] = newton;
    if (a.gmres_iters) a.gmres_iters[b] = gtotal;
    a.converged[b] = conv ? 1 : 0;
    if (a.final_mismatch) a.final_mismatch[b] = fnorm;
    if (a.work_bytes) a.work_bytes[b] = work;
  }
}

// ---------------------------------------------------------------------------
// Adjoint.  For w = [w_P on Theta ; w_Q on Q] and c = w_P + j w_Q (zero where
// undefined), w^T dF = Re sum_k g_k dV_k with g = conj(c I) + Ybus^T (c conj V),
// so (J^T w) = [-Im(g V) on Theta ; Re(g V) / |V| on Q].
template <int BLOCK, int K>
__device__ void vjp(const TxDev<double>& net, const Scen& sc, int kd, double (&w)[K], double* xs) {
  const int nth = net.nth, npq = net.npq, m = net.m;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int r = (int)row<BLOCK>(k);
    if (k < kd && r < m) xs[r] = w[k];
  }
  __syncthreads();
  auto cc = [&](int bus, double& cr, double& ci) {
    cr = bus < nth ? xs[bus] : 0.0;
    ci = bus < npq ? xs[nth + bus] : 0.0;
  };
#pragma unroll 1
  for (int k = 0; k < kd; ++k) {
    const int r = (int)row<BLOCK>(k);
    if (r < m) {
      const int i = r < nth ? r : r - nth;
      double gr = 0.0, gi = 0.0;  // (Y^T (c conj V))_i
      for (int p = net.yt_ptr[i]; p < net.yt_ptr[i + 1]; ++p) {
        const int j = net.yt_col[p];
        double cr, ci;
        cc(j, cr, ci);
        const double vr = sc.vre[j], vi = sc.vim[j];
        const double ur = cr * vr + ci * vi, ui = ci * vr - cr * vi;  // c conj(V)
        const double yr = net.yt_re[p], yi = net.yt_im[p];
        gr += yr * ur - yi * ui;
        gi += yr * ui + yi * ur;
      }
      double cr, ci;
      cc(i, cr, ci);
      const double Ir = sc.ire[i], Ii = sc.iim[i];
      gr += cr * Ir - ci * Ii;  // conj(c I)
      gi -= cr * Ii + ci * Ir;
      const double vr = sc.vre[i], vi = sc.vim[i];
      const double pr = gr * vr - gi * vi, pi = gr * vi + gi * vr;  // g V
      rset(w, k, r < nth ? -pi : pr * sc.ivm[i]);
    }
  }
  __syncthreads();
}

// z = M^-T w: z_Q = diag(|V_Q|)^-1 (B'' + eps I)^-1 w_Q,
//             z_Theta = diag(|V_Theta|)^-1 (B' + eps I)^-1 (w_Theta - G^T z_Q).
template <int BLOCK, int K>
__device__ void precond_t(const TxDev<double>& net, const Scen& sc, int kd, double (&w)[K], double* xs,
                          double* tmp) {
  const int nth = net.nth, m = net.m;
  double* x1 = xs;
  double* x2 = xs + nth;
  if (net.npq > 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int r = (int)row<BLOCK>(k);
      if (k < kd && r >= nth && r < m) x2[net.bpp.pinv[r - nth]] = w[k];
    }
    __syncthreads();
    spd_apply<double, BLOCK>(net.bpp, x2, tmp);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int r = (int)row<BLOCK>(k);
      if (k < kd && r >= nth && r < m) x2[net.bpp.pinv[r - nth]] *= sc.ivm[r - nth];
    }
    __syncthreads();
  }
#pragma unroll 1
  for (int k = 0; k < kd; ++k) {
    const int r = (int)row<BLOCK>(k);
    if (r < nth) {
      double t = rget(w, k);
      for (int p = net.gt_ptr[r]; p < net.gt_ptr[r + 1]; ++p) t -= net.gt_val[p] * x2[net.gt_col[p]];
      x1[net.bp.pinv[r]] = t;
    }
  }
  __syncthreads();
  spd_apply<double, BLOCK>(net.bp, x1, tmp);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int r = (int)row<BLOCK>(k);
    if (k < kd) {
      if (r < nth) w[k] = x1[net.bp.pinv[r]] * sc.ivm[r];
      else if (r < m) w[k] = x2[net.bpp.pinv[r - nth]];
    }
  }
  __syncthreads();
}

template <int BLOCK, int K>
__global__ __launch_bounds__(BLOCK) void adjoint_kernel(const TxDev<double>* __restrict__ netp, AdjLaunch a) {
  constexpr int NW = BLOCK / WAVE;
  extern __shared__ __align__(16) unsigned char smem[];
  const TxDev<double>& net = *netp;
  const int b = blockIdx.x;
  const int n = net.n, nth = net.nth, npq = net.npq, m = net.m;
  const int R = a.restart;
  const int kmax = net.bp.k > net.bpp.k ? net.bp.k : net.bpp.k;
  const NrLayout L = nr_layout(n, m, kmax, R, NW, 8);
  const Smem<double> s = carve<double>(smem, L);
  const int kd = ((n > m ? n : m) + BLOCK - 1) / BLOCK;
  const unsigned mp = (unsigned)kd * BLOCK;
  const Scen sc = scen_at(a.ws_d + (int64_t)b * a.ws_d_stride, n, mp);
  double* basis = a.ws_basis + (int64_t)b * a.ws_b_stride;
  const int* ext = net.int2ext;
  const double* V = a.v + 2 * (int64_t)b * a.ld;
  const double* tg = a.dl_dv + 2 * (int64_t)b * a.ld;

  // V, |V|, 1/|V| and I = Ybus V at the given voltages
  for (int i = threadIdx.x; i < n; i += BLOCK) {
    const double vr = V[2 * ext[i]], vi = V[2 * ext[i] + 1];
    const double vm = sqrt(vr * vr + vi * vi);
    sc.vre[i] = vr;
    sc.vim[i] = vi;
    sc.vm[i] = vm;
    sc.ivm[i] = 1.0 / vm;
    s.vs[2 * i] = vr;
    s.vs[2 * i + 1] = vi;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += BLOCK) {
    double Ir = 0.0, Ii = 0.0;
    for (int p = net.y_ptr[i]; p < net.y_ptr[i + 1]; ++p) {
      const int c = net.y_col[p];
      const double yr = net.y_re[p], yi = net.y_im[p], vr = s.vs[2 * c], vi = s.vs[2 * c + 1];
      Ir += yr * vr - yi * vi;
      Ii += yr * vi + yi * vr;
    }
    sc.ire[i] = Ir;
    sc.iim[i] = Ii;
  }
  // dL/dx from the torch-convention gradient t = dL/dRe V + j dL/dIm V:
  // dL/dtheta = Im(t) Re(V) - Re(t) Im(V), dL/d|V| = (Re(t) Re(V) + Im(t) Im(V)) / |V|
#pragma unroll 1
  for (int k = 0; k < kd; ++k) {
    const int r = (int)row<BLOCK>(k);
    if (r < m) {
      const int i = r < nth ? r : r - nth;
      const double tr = tg[2 * ext[i]], ti = tg[2 * ext[i] + 1];
      const double vr = V[2 * ext[i]], vi = V[2 * ext[i] + 1];
      sc.F[r] = r < nth ? ti * vr - tr * vi : (tr * vr + ti * vi) / sqrt(vr * vr + vi * vi);
    } else {
      sc.F[r] = 0.0;
    }
  }
  __syncthreads();

  auto apply_jt = [&](double (&w)[K]) { vjp<BLOCK, K>(net, sc, kd, w, s.xs); };
  auto apply_mt = [&](double (&w)[K]) { precond_t<BLOCK, K>(net, sc, kd, w, s.xs, s.tmp); };
  const ByteModel bm{8.0 * m, 8.0 * m, 8.0 * n};
  double work = 0.0;
  bool ok;
  const int its = gmres_solve<double, BLOCK, K>(apply_jt, apply_mt, sc.F, sc.dx, basis, mp, kd, R,
                                                a.max_restarts, a.rtol, s, &ok, bm, &work);
  double* gp = a.grad_p + (int64_t)b * a.ld;
  double* gq = a.grad_q + (int64_t)b * a.ld;
  // rows that carry no state (the slack's P, the Q of PV buses and the slack) are zero
  for (int i = threadIdx.x; i < n; i += BLOCK) {
    if (i >= nth) gp[ext[i]] = 0.0;
    if (i >= npq) gq[ext[i]] = 0.0;
  }
#pragma unroll 1
  for (int k = 0; k < kd; ++k) {
    const int r = (int)row<BLOCK>(k);
    if (r < nth) gp[ext[r]] = sc.dx[r];
    else if (r < m) gq[ext[r - nth]] = sc.dx[r];
  }
  if (threadIdx.x == 0) {
    if (a.gmres_iters) a.gmres_iters[b] = its;
    if (a.converged) a.converged[b] = ok ? 1 : 0;
  }
}

// Shapes: BLOCK threads, K rows per thread, max(n, m) <= BLOCK * K.
template <typename Launch>
void dispatch_shape(int rows, Launch&& go) {
  if (rows <= 64) go.template operator()<64, 1>();
  else if (rows <= 256) go.template operator()<64, 4>();
  else if (rows <= 1024) go.template operator()<256, 4>();
  else if (rows <= 4096) go.template operator()<256, 16>();
  else if (rows <= 16384) go.template operator()<512, 32>();
  else fail(PF_INVALID_ARG, "networks above 16384 state rows are not supported");
}

struct ShapeOf {
  int* block;
  template <int BLOCK, int K>
  void operator()() const {
    *block = BLOCK;
  }
};

size_t lds_bytes(const TxNetwork& net, int R, int block, int ts) {
  const int kmax = std::max(net.bp.host.k, net.bpp.host.k);
  const NrLayout L = nr_layout(net.n, net.m, kmax, R, block / WAVE, ts);
  if (L.total > 160 * 1024)
    fail(PF_INVALID_ARG, "network too large for the per-scenario LDS layout (" + std::to_string(L.total) +
                             " bytes)");
  return (size_t)L.total;
}

template <typename T>
struct NrGo {
  const TxNetwork& net;
  const NRLaunch& a;
  hipStream_t s;
  template <int BLOCK, int K>
  void operator()() const {
    const size_t lds = lds_bytes(net, a.restart, BLOCK, (int)sizeof(T));
    auto kernel = nr_kernel<T, BLOCK, K>;
    if (lds > 64 * 1024)
      PFX_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(kernel, dim3(a.batch), dim3(BLOCK), lds, s, net.desc<T>(), a);
    PFX_HIP(hipGetLastError());
  }
};

struct AdjGo {
  const TxNetwork& net;
  const AdjLaunch& a;
  hipStream_t s;
  template <int BLOCK, int K>
  void operator()() const {
    const size_t lds = lds_bytes(net, a.restart, BLOCK, 8);
    auto kernel = adjoint_kernel<BLOCK, K>;
    if (lds > 64 * 1024)
      PFX_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(kernel, dim3(a.batch), dim3(BLOCK), lds, s, net.desc<double>(), a);
    PFX_HIP(hipGetLastError());
  }
};

}  // namespace

int64_t nr_padded_rows(const TxNetwork& net) {
  const int rows = std::max(net.n, net.m);
  int block = 0;
  dispatch_shape(rows, ShapeOf{&block});
  return (int64_t)((rows + block - 1) / block) * block;
}
int64_t nr_ws_doubles(const TxNetwork& net) { return 7 * (int64_t)net.n + 2 * nr_padded_rows(net); }
int64_t adj_ws_doubles(const TxNetwork& net) { return nr_ws_doubles(net); }

void launch_nr(const TxNetwork& net, bool mixed, const NRLaunch& a, hipStream_t s) {
  if (a.batch == 0) return;
  const int rows = std::max(net.n, net.m);
  if (mixed) dispatch_shape(rows, NrGo<float>{net, a, s});
  else dispatch_shape(rows, NrGo<double>{net, a, s});
}

void launch_adjoint(const TxNetwork& net, const AdjLaunch& a, hipStream_t s) {
  if (a.batch == 0) return;
  dispatch_shape(std::max(net.n, net.m), AdjGo{net, a, s});
}

// ---------------------------------------------------------------------------
// Branch-current loss L = sum_f |I_f|^2, I_f = (y_s + j b/2) V_f - y_s V_t,
// and dL/dV in torch's convention conj(g), g_k = dL/dV_k (complex derivative).
// One workgroup per scenario; the gradient is accumulated per bus by walking
// each bus's incident branches (no atomics, fixed order).
__global__ __launch_bounds__(256) void branch_loss_kernel(const TxDev<double>* __restrict__ netp,
                                                          const int* inc_ptr, const int* inc_br, LossLaunch a) {
  __shared__ double red[4];
  const TxDev<double>& net = *netp;
  const int b = blockIdx.x;
  const double* v = a.v + 2 * (int64_t)b * a.ld;
  const int* ext = net.int2ext;
  double acc = 0.0;
  for (int k = threadIdx.x; k < net.n_branch; k += 256) {
    const int f = ext[net.br_f[k]], t = ext[net.br_t[k]];
    const double ysr = net.br_ys_re[k], ysi = net.br_ys_im[k], hb = 0.5 * net.br_b[k];
    const double vfr = v[2 * f], vfi = v[2 * f + 1], vtr = v[2 * t], vti = v[2 * t + 1];
    const double ir = ysr * vfr - (ysi + hb) * vfi - (ysr * vtr - ysi * vti);
    const double ii = ysr * vfi + (ysi + hb) * vfr - (ysr * vti + ysi * vtr);
    acc += ir * ir + ii * ii;
  }
  const double tot = block_sum<double, 256>(acc, red);
  if (threadIdx.x == 0) a.loss[b] = tot;
  if (!a.dl_dv) return;
  double* gout = a.dl_dv + 2 * (int64_t)b * a.ld;
  for (int i = threadIdx.x; i < net.n; i += 256) {
    double gr = 0.0, gi = 0.0;  // torch gradient dL/dRe + j dL/dIm = 2 sum I_f conj(coef)
    for (int q = inc_ptr[i]; q < inc_ptr[i + 1]; ++q) {
      const int k = inc_br[q];
      const int f = ext[net.br_f[k]], t = ext[net.br_t[k]];
      const double ysr = net.br_ys_re[k], ysi = net.br_ys_im[k], hb = 0.5 * net.br_b[k];
      const double vfr = v[2 * f], vfi = v[2 * f + 1], vtr = v[2 * t], vti = v[2 * t + 1];
      const double ir = ysr * vfr - (ysi + hb) * vfi - (ysr * vtr - ysi * vti);
      const double ii = ysr * vfi + (ysi + hb) * vfr - (ysr * vti + ysi * vtr);
      // coefficient of V_i in I_f: y_s + j b/2 at the from end, -y_s at the to end
      double cr, ci;
      if (net.br_f[k] == i) {
        cr = ysr;
        ci = ysi + hb;
      } else {
        cr = -ysr;
        ci = -ysi;
      }
      gr += 2.0 * (cr * ir + ci * ii);
      gi += 2.0 * (cr * ii - ci * ir);
    }
    const int e = ext[i];
    gout[2 * e] = gr;
    gout[2 * e + 1] = gi;
  }
}

void launch_branch_loss(const TxNetwork& net, const LossLaunch& a, hipStream_t s) {
  if (a.batch == 0) return;
  hipLaunchKernelGGL(branch_loss_kernel, dim3(a.batch), dim3(256), 0, s, net.desc<double>(),
                     net.inc_ptr.as<int>(), net.inc_br.as<int>(), a);
  PFX_HIP(hipGetLastError());
}

}  // namespace pfx
