// Batched Newton-Raphson power flow for meshed grids (Sec. II-A), one
// workgroup per scenario.
//
// A workgroup owns one scenario for its whole solve: every vector of length n
// (buses) or m = |Theta| + |Q| (Newton state) is split over the workgroup's
// threads by rows (thread t owns rows t, t + BLOCK, ...), so per-scenario dot
// products and norms are workgroup reductions and no grid-wide
// synchronisation is ever needed.  Per-scenario data:
//   * LDS: the vector being gathered (V for Ybus V, the direction for the
//     Jacobian-vector product, the preconditioner's work vector) and the small
//     GMRES matrices;
//   * registers: the current Krylov vector w and the Newton step dx;
//   * HBM (scenario-major workspace): theta, |V|, V, I, F and the Krylov basis,
//     always accessed at the thread's own rows, so consecutive lanes touch
//     consecutive addresses.
// The shared network data (Ybus, factors of B' and B'') is read through the
// caches by every workgroup.
//
// Steps per Newton iteration (eqs. (1)-(3), (7)-(9)):
//   mismatch  V = |V| e^{j theta}, I = Ybus V, S = V conj(I),
//             F = [Re S - P on Theta ; Im S - Q on Q], max |F|
//   GMRES     left-preconditioned restarted GMRES on J dx = -F with
//             Jacobian-vector products dS = dV conj(I) + V conj(Ybus dV),
//             dV = V (j dtheta + d|V| / |V|), the preconditioner applied by
//             forward block substitution, classical Gram-Schmidt with one
//             re-orthogonalisation, Givens rotations on the Hessenberg matrix
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

// Workgroup sum; every thread gets the result.  Ends with a barrier so `red`
// can be reused right away.
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

struct NrLayout {
  int xs, tmp, H, cs, sn, y, g, h1, h2, red, misc, total;
};

__host__ __device__ inline int align16(int x) { return (x + 15) & ~15; }

__host__ __device__ inline NrLayout nr_layout(int n, int m, int kmax, int R, int NW, int ts) {
  NrLayout L;
  int o = 0;
  const int xs_bytes = m * ts > 2 * n * 8 ? m * ts : 2 * n * 8;
  L.xs = o;   o += align16(xs_bytes);
  L.tmp = o;  o += align16((kmax > 0 ? kmax : 1) * ts);
  L.H = o;    o += align16((R + 1) * R * ts);
  L.cs = o;   o += align16(R * ts);
  L.sn = o;   o += align16(R * ts);
  L.y = o;    o += align16(R * ts);
  L.g = o;    o += align16((R + 1) * ts);
  L.h1 = o;   o += align16((R + 1) * ts);
  L.h2 = o;   o += align16((R + 1) * ts);
  const int red_bytes = (R + 1) * NW * ts > NW * 8 ? (R + 1) * NW * ts : NW * 8;
  L.red = o;  o += align16(red_bytes);
  L.misc = o; o += 64;
  L.total = o;
  return L;
}

// ---------------------------------------------------------------------------
// Solve (B + eps I) x = b in place for the vector held in LDS in factor order
// (see factor.hpp).  Ends with a barrier.
// The factor is A = L D L^T with unit lower L over the sparse prefix and the
// explicit inverse of the Schur complement S over the dense core:
//   y1 = L11^-1 b1 (levels), t = b2 - L21 y1, x2 = S^-1 t, w1 = D11^-1 y1,
//   x1 = L11^-T (w1 - L21^T x2) (levels, reverse order).
template <typename T, int BLOCK>
__device__ void spd_apply(const SpdDev<T>& f, T* xs, T* tmp) {
  for (int l = 0; l < f.nfl; ++l) {
    const int s = f.f_lev[l], e = f.f_lev[l + 1];
    for (int q = s + (int)threadIdx.x; q < e; q += BLOCK) {
      const int i = f.f_rows[q];
      T a = xs[i];
      for (int p = f.L_ptr[i]; p < f.L_ptr[i + 1]; ++p) a -= f.L_val[p] * xs[f.L_col[p]];
      xs[i] = a;
    }
    __syncthreads();
  }
  if (f.k > 0) {
    for (int i = f.c + (int)threadIdx.x; i < f.N; i += BLOCK) {
      T a = xs[i];
      for (int p = f.L_ptr[i]; p < f.L_ptr[i + 1]; ++p) a -= f.L_val[p] * xs[f.L_col[p]];
      tmp[i - f.c] = a;
    }
    __syncthreads();
    for (int i = (int)threadIdx.x; i < f.k; i += BLOCK) {
      T a = 0;
      const T* col = f.Sinv + i;
      for (int l = 0; l < f.k; ++l) a += col[(size_t)l * f.k] * tmp[l];
      xs[f.c + i] = a;
    }
  }
  for (int j = (int)threadIdx.x; j < f.c; j += BLOCK) xs[j] *= f.dinv[j];
  __syncthreads();
  for (int l = 0; l < f.nbl; ++l) {
    const int s = f.b_lev[l], e = f.b_lev[l + 1];
    for (int q = s + (int)threadIdx.x; q < e; q += BLOCK) {
      const int j = f.b_rows[q];
      T a = xs[j];
      for (int p = f.T_ptr[j]; p < f.T_ptr[j + 1]; ++p) a -= f.T_val[p] * xs[f.T_col[p]];
      xs[j] = a;
    }
    __syncthreads();
  }
}

// Per-scenario views into the workspace.
struct Scen {
  double* th;   // [n] angle
  double* vm;   // [n] magnitude
  double* vre;  // [n] V
  double* vim;
  double* ire;  // [n] I = Ybus V
  double* iim;
  double* F;    // [m] mismatch
};

// z = M^-1 w for the left preconditioner of eq. (7), by the forward block
// substitution of eqs. (8)-(9):
//   z_Theta = (B' + eps I)^-1 diag(|V_Theta|)^-1 w_Theta
//   z_Q     = (B'' + eps I)^-1 diag(|V_Q|)^-1 (w_Q - G z_Theta)
template <typename T, int BLOCK, int K>
__device__ void precond(const TxDev<T>& net, const double* vm, T (&w)[K], T* xs, T* tmp) {
  T* x1 = xs;
  T* x2 = xs + net.nth;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int r = threadIdx.x + k * BLOCK;
    if (r < net.nth) x1[net.bp.pinv[r]] = w[k] / (T)vm[r];
  }
  __syncthreads();
  spd_apply<T, BLOCK>(net.bp, x1, tmp);
  if (net.npq > 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int r = threadIdx.x + k * BLOCK;
      if (r >= net.nth && r < net.m) {
        const int q = r - net.nth;
        T t = w[k];
        for (int p = net.g_ptr[q]; p < net.g_ptr[q + 1]; ++p) t -= net.g_val[p] * x1[net.g_col[p]];
        x2[net.bpp.pinv[q]] = t / (T)vm[q];
      }
    }
    __syncthreads();
    spd_apply<T, BLOCK>(net.bpp, x2, tmp);
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int r = threadIdx.x + k * BLOCK;
    if (r < net.nth) w[k] = x1[net.bp.pinv[r]];
    else if (r < net.m) w[k] = x2[net.bpp.pinv[r - net.nth]];
  }
  __syncthreads();
}

// w <- J w, the Jacobian of the mismatch at the current V (with I = Ybus V).
template <typename T, int BLOCK, int K>
__device__ void jvp(const TxDev<T>& net, const Scen& sc, T (&w)[K], T* xs) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int r = threadIdx.x + k * BLOCK;
    if (r < net.m) xs[r] = w[k];
  }
  __syncthreads();
  const int nth = net.nth, npq = net.npq;
  auto dv = [&](int bus, T& dr, T& di) {
    const T pth = bus < nth ? xs[bus] : (T)0;
    const T pv = bus < npq ? xs[nth + bus] : (T)0;
    const T vr = (T)sc.vre[bus], vi = (T)sc.vim[bus];
    const T a = pv / (T)sc.vm[bus];
    dr = vr * a - vi * pth;
    di = vi * a + vr * pth;
  };
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int r = threadIdx.x + k * BLOCK;
    if (r < net.m) {
      const int i = r < nth ? r : r - nth;
      T dIr = 0, dIi = 0;
      for (int p = net.y_ptr[i]; p < net.y_ptr[i + 1]; ++p) {
        T dr, di;
        dv(net.y_col[p], dr, di);
        const T yr = (T)net.y_re[p], yi = (T)net.y_im[p];
        dIr += yr * dr - yi * di;
        dIi += yr * di + yi * dr;
      }
      T dVr, dVi;
      dv(i, dVr, dVi);
      const T Ir = (T)sc.ire[i], Ii = (T)sc.iim[i];
      const T vr = (T)sc.vre[i], vi = (T)sc.vim[i];
      // dS = dV conj(I) + V conj(dI)
      w[k] = r < nth ? dVr * Ir + dVi * Ii + vr * dIr + vi * dIi
                     : dVi * Ir - dVr * Ii + vi * dIr - vr * dIi;
    }
  }
  __syncthreads();
}

// h[i] = <basis_i, w> for i < nv (results in LDS h; ends with a barrier).
template <typename T, int BLOCK, int K>
__device__ void multi_dot(const T* basis, int64_t stride, int nv, int m, const T (&w)[K], T* red, T* h) {
  constexpr int NW = BLOCK / WAVE;
  for (int i = 0; i < nv; ++i) {
    const T* v = basis + i * stride;
    T acc = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int r = threadIdx.x + k * BLOCK;
      if (r < m) acc += v[r] * w[k];
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & (WAVE - 1)) == 0) red[i * NW + threadIdx.x / WAVE] = acc;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nv; i += BLOCK) {
    T s = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) s += red[i * NW + q];
    h[i] = s;
  }
  __syncthreads();
}

// w -= sum_i h[i] basis_i
template <typename T, int BLOCK, int K>
__device__ void subtract_proj(const T* basis, int64_t stride, int nv, int m, T (&w)[K], const T* h) {
  for (int i = 0; i < nv; ++i) {
    const T hi = h[i];
    const T* v = basis + i * stride;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int r = threadIdx.x + k * BLOCK;
      if (r < m) w[k] -= hi * v[r];
    }
  }
}

// Mismatch at the current (theta, |V|): writes V, I and F to the workspace and
// returns max |F| (NaN if any entry is NaN).
template <int BLOCK, int K>
__device__ double mismatch(const TxDev<double>& ynet, int n, int nth, int npq, int m, const Scen& sc,
                           const double* P, const double* Q, const int* int2ext, double* vs,
                           double* red) {
  for (int i = threadIdx.x; i < n; i += BLOCK) {
    double s, c;
    sincos(sc.th[i], &s, &c);
    const double vr = sc.vm[i] * c, vi = sc.vm[i] * s;
    sc.vre[i] = vr;
    sc.vim[i] = vi;
    vs[2 * i] = vr;
    vs[2 * i + 1] = vi;
  }
  __syncthreads();
  double fmax = 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int r = threadIdx.x + k * BLOCK;
    if (r < m) {
      const int i = r < nth ? r : r - nth;
      double Ir = 0.0, Ii = 0.0;
      for (int p = ynet.y_ptr[i]; p < ynet.y_ptr[i + 1]; ++p) {
        const int c = ynet.y_col[p];
        const double yr = ynet.y_re[p], yi = ynet.y_im[p];
        const double vr = vs[2 * c], vi = vs[2 * c + 1];
        Ir += yr * vr - yi * vi;
        Ii += yr * vi + yi * vr;
      }
      const double vr = vs[2 * i], vi = vs[2 * i + 1];
      double f;
      if (r < nth) {
        sc.ire[i] = Ir;
        sc.iim[i] = Ii;
        f = vr * Ir + vi * Ii - P[int2ext[i]];
      } else {
        f = vi * Ir - vr * Ii - Q[int2ext[i]];
      }
      sc.F[r] = f;
      fmax = nanmax(fmax, fabs(f));
    }
  }
  return block_nanmax<BLOCK>(fmax, red);
}

// LDS carve-up shared by the NR and adjoint kernels.
template <typename T>
struct Smem {
  T* xs;
  double* vs;
  T* tmp;
  T* H;  // column-major, leading dimension R + 1
  T* cs;
  T* sn;
  T* yv;
  T* g;
  T* h1;
  T* h2;
  T* red;
  double* redd;
  T* misc;
};

template <typename T>
__device__ Smem<T> carve(unsigned char* smem, const NrLayout& L) {
  Smem<T> s;
  s.xs = reinterpret_cast<T*>(smem + L.xs);
  s.vs = reinterpret_cast<double*>(smem + L.xs);
  s.tmp = reinterpret_cast<T*>(smem + L.tmp);
  s.H = reinterpret_cast<T*>(smem + L.H);
  s.cs = reinterpret_cast<T*>(smem + L.cs);
  s.sn = reinterpret_cast<T*>(smem + L.sn);
  s.yv = reinterpret_cast<T*>(smem + L.y);
  s.g = reinterpret_cast<T*>(smem + L.g);
  s.h1 = reinterpret_cast<T*>(smem + L.h1);
  s.h2 = reinterpret_cast<T*>(smem + L.h2);
  s.red = reinterpret_cast<T*>(smem + L.red);
  s.redd = reinterpret_cast<double*>(smem + L.red);
  s.misc = reinterpret_cast<T*>(smem + L.misc);
  return s;
}

// Restarted GMRES with left preconditioning for A x = b from x = 0, where
// apply_a(w) overwrites w with A w and apply_m(w) with M^-1 w (both on the
// thread's own rows).  b is read from `rhs` (FP64, own rows); x accumulates in
// FP64.  Stops when ||M^-1 (b - A x)|| <= rtol ||M^-1 b|| (the Givens estimate
// inside a cycle), after max_restarts cycles, or at a breakdown.  Returns the
// number of Arnoldi steps; *converged tells whether the tolerance was met.
// Orthogonalisation: classical Gram-Schmidt with one re-orthogonalisation.
// Algorithmic HBM bytes of one scenario (the byte model reported with the
// solve): with w = sizeof(T), per Jacobian-vector product 2 w m + 32 n, per
// preconditioner application 2 w m + 8 n, per Arnoldi step j (orthogonalising
// against j + 1 vectors by CGS2) (4 j + 6) w m, per cycle end (k + 2) w m, per
// cycle start 8 m + w m, per mismatch evaluation 32 n + 16 m and per Newton
// update 16 m.
struct ByteModel {
  double wm, m8, n8;
  __device__ double jvp() const { return 2 * wm + 4 * n8; }
  __device__ double pre() const { return 2 * wm + n8; }
  __device__ double orth(int j) const { return (4.0 * j + 6.0) * wm; }
  __device__ double mismatch() const { return 4 * n8 + 2 * m8; }
  __device__ double update() const { return 2 * m8; }
};

template <typename T, int BLOCK, int K, typename ApplyA, typename ApplyM>
__device__ int gmres_solve(ApplyA&& apply_a, ApplyM&& apply_m, const double* rhs, T* basis, int m, int R,
                           int max_restarts, T rtol, double (&x)[K], const Smem<T>& s, bool* converged,
                           const ByteModel& bm, double* work) {
  T w[K];
  T beta0 = 0;
  int total = 0;
  bool done = false;
#pragma unroll
  for (int k = 0; k < K; ++k) x[k] = 0.0;
  for (int cycle = 0; cycle < max_restarts && !done; ++cycle) {
    *work += (cycle > 0 ? bm.jvp() : 0.0) + bm.pre() + bm.m8 + bm.wm;
    if (cycle == 0) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int r = threadIdx.x + k * BLOCK;
        w[k] = r < m ? (T)rhs[r] : (T)0;
      }
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k) w[k] = (T)x[k];
      apply_a(w);
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int r = threadIdx.x + k * BLOCK;
        w[k] = r < m ? (T)rhs[r] - w[k] : (T)0;
      }
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
      const int r = threadIdx.x + k * BLOCK;
      w[k] *= ib;
      if (r < m) basis[r] = w[k];
    }
    if (threadIdx.x == 0) s.g[0] = beta;
    int steps = 0;
    T res = beta;
    for (int j = 0; j < R; ++j) {
      apply_a(w);
      apply_m(w);
      *work += bm.jvp() + bm.pre() + bm.orth(j);
      multi_dot<T, BLOCK, K>(basis, m, j + 1, m, w, s.red, s.h1);
      subtract_proj<T, BLOCK, K>(basis, m, j + 1, m, w, s.h1);
      multi_dot<T, BLOCK, K>(basis, m, j + 1, m, w, s.red, s.h2);
      subtract_proj<T, BLOCK, K>(basis, m, j + 1, m, w, s.h2);
      T s2 = 0;
#pragma unroll
      for (int k = 0; k < K; ++k) s2 += w[k] * w[k];
      const T hn = sqrt(block_sum<T, BLOCK>(s2, s.red));
      if (threadIdx.x == 0) {
        T* Hj = s.H + j * (R + 1);
        for (int i = 0; i <= j; ++i) Hj[i] = s.h1[i] + s.h2[i];
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
      T* vnext = basis + (int64_t)(j + 1) * m;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int r = threadIdx.x + k * BLOCK;
        w[k] *= ih;
        if (r < m) vnext[r] = w[k];
      }
    }
    total += steps;
    *work += (steps + 2) * bm.wm;
    // y = H^-1 g (upper triangular after the rotations)
    if (threadIdx.x == 0) {
      for (int i = steps - 1; i >= 0; --i) {
        T a = s.g[i];
        for (int l = i + 1; l < steps; ++l) a -= s.H[l * (R + 1) + i] * s.yv[l];
        const T d = s.H[i * (R + 1) + i];
        s.yv[i] = d != (T)0 ? a / d : (T)0;
      }
    }
    __syncthreads();
    for (int i = 0; i < steps; ++i) {
      const double yi = (double)s.yv[i];
      const T* v = basis + (int64_t)i * m;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int r = threadIdx.x + k * BLOCK;
        if (r < m) x[k] += yi * (double)v[r];
      }
    }
    done = !(res > rtol * beta0);
    __syncthreads();
  }
  *converged = done;
  return total;
}

template <typename T, int BLOCK, int K>
__global__ __launch_bounds__(BLOCK) void nr_kernel(TxDev<double> ynet, TxDev<T> net, NRLaunch a) {
  constexpr int NW = BLOCK / WAVE;
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = blockIdx.x;
  const int n = net.n, nth = net.nth, npq = net.npq, m = net.m;
  const int R = a.restart;
  const int kmax = net.bp.k > net.bpp.k ? net.bp.k : net.bpp.k;
  const NrLayout L = nr_layout(n, m, kmax, R, NW, (int)sizeof(T));
  const Smem<T> s = carve<T>(smem, L);

  double* ws = a.ws_d + (int64_t)b * a.ws_d_stride;
  const Scen sc{ws, ws + n, ws + 2 * n, ws + 3 * n, ws + 4 * n, ws + 5 * n, ws + 6 * n};
  T* basis = reinterpret_cast<T*>(a.ws_basis) + (int64_t)b * a.ws_b_stride;
  const double* P = a.p_inj + (int64_t)b * a.ld;
  const double* Q = a.q_inj + (int64_t)b * a.ld;
  const double* VS = a.vm_set + (int64_t)b * a.ld;
  const int* int2ext = ynet.int2ext;

  // flat start: theta = 0, |V| = set-point at PV and slack, 1 at PQ buses
  for (int i = threadIdx.x; i < n; i += BLOCK) {
    sc.th[i] = 0.0;
    sc.vm[i] = i < npq ? 1.0 : VS[int2ext[i]];
  }
  __syncthreads();

  auto apply_j = [&](T (&w)[K]) { jvp<T, BLOCK, K>(net, sc, w, s.xs); };
  auto apply_m = [&](T (&w)[K]) { precond<T, BLOCK, K>(net, sc.vm, w, s.xs, s.tmp); };

  int newton = 0, gtotal = 0;
  bool conv = false;
  double fnorm = 0.0;
  const ByteModel bm{(double)sizeof(T) * m, 8.0 * m, 8.0 * n};
  double work = 0.0;
  for (;;) {
    work += bm.mismatch();
    fnorm = mismatch<BLOCK, K>(ynet, n, nth, npq, m, sc, P, Q, int2ext, s.vs, s.redd);
    if (!(fnorm <= a.diverge)) break;
    if (fnorm <= a.tol) {
      conv = true;
      break;
    }
    if (newton >= a.max_newton) break;
    // right-hand side -F in place
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int r = threadIdx.x + k * BLOCK;
      if (r < m) sc.F[r] = -sc.F[r];
    }
    double dx[K];
    bool lin_ok;
    gtotal += gmres_solve<T, BLOCK, K>(apply_j, apply_m, sc.F, basis, m, R, a.max_restarts, (T)a.rtol,
                                       dx, s, &lin_ok, bm, &work);
    work += bm.update();
    // Newton update (eq. (3)), FP64
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int r = threadIdx.x + k * BLOCK;
      if (r < nth) sc.th[r] += dx[k];
      else if (r < m) sc.vm[r - nth] += dx[k];
    }
    __syncthreads();
    ++newton;
  }

  double* vout = a.v_out + 2 * (int64_t)b * a.ld;
  for (int i = threadIdx.x; i < n; i += BLOCK) {
    const int e = int2ext[i];
    vout[2 * e] = sc.vre[i];
    vout[2 * e + 1] = sc.vim[i];
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
__device__ void vjp(const TxDev<double>& net, const Scen& sc, const int* yt_ptr, const int* yt_col,
                    const double* yt_re, const double* yt_im, double (&w)[K], double* xs) {
  const int nth = net.nth, npq = net.npq;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int r = threadIdx.x + k * BLOCK;
    if (r < net.m) xs[r] = w[k];
  }
  __syncthreads();
  auto cc = [&](int bus, double& cr, double& ci) {
    cr = bus < nth ? xs[bus] : 0.0;
    ci = bus < npq ? xs[nth + bus] : 0.0;
  };
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int r = threadIdx.x + k * BLOCK;
    if (r < net.m) {
      const int i = r < nth ? r : r - nth;
      double gr = 0.0, gi = 0.0;  // (Y^T (c conj V))_i
      for (int p = yt_ptr[i]; p < yt_ptr[i + 1]; ++p) {
        const int j = yt_col[p];
        double cr, ci;
        cc(j, cr, ci);
        const double vr = sc.vre[j], vi = sc.vim[j];
        const double ur = cr * vr + ci * vi, ui = ci * vr - cr * vi;  // c conj(V)
        const double yr = yt_re[p], yi = yt_im[p];
        gr += yr * ur - yi * ui;
        gi += yr * ui + yi * ur;
      }
      double cr, ci;
      cc(i, cr, ci);
      const double Ir = sc.ire[i], Ii = sc.iim[i];
      gr += cr * Ir - ci * Ii;     // conj(c I)
      gi -= cr * Ii + ci * Ir;
      const double vr = sc.vre[i], vi = sc.vim[i];
      const double pr = gr * vr - gi * vi, pi = gr * vi + gi * vr;  // g V
      w[k] = r < nth ? -pi : pr / sc.vm[i];
    }
  }
  __syncthreads();
}

// z = M^-T w: z_Q = diag(|V_Q|)^-1 (B'' + eps I)^-1 w_Q,
//             z_Theta = diag(|V_Theta|)^-1 (B' + eps I)^-1 (w_Theta - G^T z_Q).
template <int BLOCK, int K>
__device__ void precond_t(const TxDev<double>& net, const double* vm, double (&w)[K], double* xs, double* tmp) {
  double* x1 = xs;
  double* x2 = xs + net.nth;
  if (net.npq > 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int r = threadIdx.x + k * BLOCK;
      if (r >= net.nth && r < net.m) x2[net.bpp.pinv[r - net.nth]] = w[k];
    }
    __syncthreads();
    spd_apply<double, BLOCK>(net.bpp, x2, tmp);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int r = threadIdx.x + k * BLOCK;
      if (r >= net.nth && r < net.m) x2[net.bpp.pinv[r - net.nth]] /= vm[r - net.nth];
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int r = threadIdx.x + k * BLOCK;
    if (r < net.nth) {
      double t = w[k];
      for (int p = net.gt_ptr[r]; p < net.gt_ptr[r + 1]; ++p) t -= net.gt_val[p] * x2[net.gt_col[p]];
      x1[net.bp.pinv[r]] = t;
    }
  }
  __syncthreads();
  spd_apply<double, BLOCK>(net.bp, x1, tmp);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int r = threadIdx.x + k * BLOCK;
    if (r < net.nth) w[k] = x1[net.bp.pinv[r]] / vm[r];
    else if (r < net.m) w[k] = x2[net.bpp.pinv[r - net.nth]];
  }
  __syncthreads();
}

template <int BLOCK, int K>
__global__ __launch_bounds__(BLOCK) void adjoint_kernel(TxDev<double> net, const int* yt_ptr, const int* yt_col,
                                                        const double* yt_re, const double* yt_im, AdjLaunch a) {
  constexpr int NW = BLOCK / WAVE;
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = blockIdx.x;
  const int n = net.n, nth = net.nth, npq = net.npq, m = net.m;
  const int R = a.restart;
  const int kmax = net.bp.k > net.bpp.k ? net.bp.k : net.bpp.k;
  const NrLayout L = nr_layout(n, m, kmax, R, NW, 8);
  const Smem<double> s = carve<double>(smem, L);
  double* ws = a.ws_d + (int64_t)b * a.ws_d_stride;
  const Scen sc{ws, ws + n, ws + 2 * n, ws + 3 * n, ws + 4 * n, ws + 5 * n, ws + 6 * n};
  double* basis = a.ws_basis + (int64_t)b * a.ws_b_stride;
  const int* ext = net.int2ext;
  const double* V = a.v + 2 * (int64_t)b * a.ld;
  const double* tg = a.dl_dv + 2 * (int64_t)b * a.ld;

  // V, |V| and I = Ybus V at the given voltages
  for (int i = threadIdx.x; i < n; i += BLOCK) {
    const double vr = V[2 * ext[i]], vi = V[2 * ext[i] + 1];
    sc.vre[i] = vr;
    sc.vim[i] = vi;
    sc.vm[i] = sqrt(vr * vr + vi * vi);
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
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int r = threadIdx.x + k * BLOCK;
    if (r < m) {
      const int i = r < nth ? r : r - nth;
      const double tr = tg[2 * ext[i]], ti = tg[2 * ext[i] + 1];
      const double vr = V[2 * ext[i]], vi = V[2 * ext[i] + 1];
      sc.F[r] = r < nth ? ti * vr - tr * vi : (tr * vr + ti * vi) / sqrt(vr * vr + vi * vi);
    }
  }
  __syncthreads();

  auto apply_jt = [&](double (&w)[K]) { vjp<BLOCK, K>(net, sc, yt_ptr, yt_col, yt_re, yt_im, w, s.xs); };
  auto apply_mt = [&](double (&w)[K]) { precond_t<BLOCK, K>(net, sc.vm, w, s.xs, s.tmp); };
  double lam[K];
  bool ok;
  const ByteModel bm{8.0 * m, 8.0 * m, 8.0 * n};
  double work = 0.0;
  const int its = gmres_solve<double, BLOCK, K>(apply_jt, apply_mt, sc.F, basis, m, R, a.max_restarts, a.rtol,
                                                lam, s, &ok, bm, &work);
  double* gp = a.grad_p + (int64_t)b * a.ld;
  double* gq = a.grad_q + (int64_t)b * a.ld;
  // zero the rows that carry no state (the slack's P, the Q of PV buses and the slack)
  for (int i = threadIdx.x; i < n; i += BLOCK) {
    if (i >= nth) gp[ext[i]] = 0.0;
    if (i >= npq) gq[ext[i]] = 0.0;
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int r = threadIdx.x + k * BLOCK;
    if (r < nth) gp[ext[r]] = lam[k];
    else if (r < m) gq[ext[r - nth]] = lam[k];
  }
  if (threadIdx.x == 0) {
    if (a.gmres_iters) a.gmres_iters[b] = its;
    if (a.converged) a.converged[b] = ok ? 1 : 0;
  }
}

// Supported (BLOCK, K) shapes: rows per thread K, max(n, m) <= BLOCK * K.
struct Shape {
  int block, k;
};
constexpr Shape kShapes[] = {{64, 1}, {64, 4}, {256, 4}, {256, 16}, {512, 32}};

template <typename T>
void launch_nr_t(const TxNetwork& net, const NRLaunch& a, hipStream_t s) {
  const int rows = std::max(net.n, net.m);
  const int kmax = std::max(net.bp.host.k, net.bpp.host.k);
  auto go = [&](auto kernel, int block) {
    const NrLayout L = nr_layout(net.n, net.m, kmax, a.restart, block / WAVE, (int)sizeof(T));
    if (L.total > 160 * 1024)
      fail(PF_INVALID_ARG, "network too large for the per-scenario LDS layout (" +
                               std::to_string(L.total) + " bytes)");
    if (L.total > 64 * 1024)
      PFX_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, L.total));
    hipLaunchKernelGGL(kernel, dim3(a.batch), dim3(block), L.total, s, net.view<double>(),
                       net.view<T>(), a);
    PFX_HIP(hipGetLastError());
  };
  if (rows <= 64) go(nr_kernel<T, 64, 1>, 64);
  else if (rows <= 256) go(nr_kernel<T, 64, 4>, 64);
  else if (rows <= 1024) go(nr_kernel<T, 256, 4>, 256);
  else if (rows <= 4096) go(nr_kernel<T, 256, 16>, 256);
  else if (rows <= 16384) go(nr_kernel<T, 512, 32>, 512);
  else fail(PF_INVALID_ARG, "networks above 16384 state rows are not supported");
}

}  // namespace

int64_t nr_ws_doubles(const TxNetwork& net) { return 6 * (int64_t)net.n + net.m; }
int64_t adj_ws_doubles(const TxNetwork& net) { return 6 * (int64_t)net.n + net.m; }

void launch_adjoint(const TxNetwork& net, const AdjLaunch& a, hipStream_t s) {
  if (a.batch == 0) return;
  const int rows = std::max(net.n, net.m);
  const int kmax = std::max(net.bp.host.k, net.bpp.host.k);
  auto go = [&](auto kernel, int block) {
    const NrLayout L = nr_layout(net.n, net.m, kmax, a.restart, block / WAVE, 8);
    if (L.total > 160 * 1024)
      fail(PF_INVALID_ARG, "network too large for the per-scenario LDS layout");
    if (L.total > 64 * 1024)
      PFX_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, L.total));
    hipLaunchKernelGGL(kernel, dim3(a.batch), dim3(block), L.total, s, net.view<double>(),
                       net.yt_ptr.as<int>(), net.yt_col.as<int>(), net.yt_re.as<double>(),
                       net.yt_im.as<double>(), a);
    PFX_HIP(hipGetLastError());
  };
  if (rows <= 64) go(adjoint_kernel<64, 1>, 64);
  else if (rows <= 256) go(adjoint_kernel<64, 4>, 64);
  else if (rows <= 1024) go(adjoint_kernel<256, 4>, 256);
  else if (rows <= 4096) go(adjoint_kernel<256, 16>, 256);
  else if (rows <= 16384) go(adjoint_kernel<512, 32>, 512);
  else fail(PF_INVALID_ARG, "networks above 16384 state rows are not supported");
}

void launch_nr(const TxNetwork& net, bool mixed, const NRLaunch& a, hipStream_t s) {
  if (a.batch == 0) return;
  if (mixed) launch_nr_t<float>(net, a, s);
  else launch_nr_t<double>(net, a, s);
}

// ---------------------------------------------------------------------------
// Branch-current loss L = sum_f |I_f|^2, I_f = (y_s + j b/2) V_f - y_s V_t,
// and dL/dV in torch's convention conj(g), g_k = dL/dV_k (complex derivative).
// One workgroup per scenario; the gradient is accumulated per bus by walking
// each bus's incident branches (no atomics, fixed order).
__global__ __launch_bounds__(256) void branch_loss_kernel(TxDev<double> net, const int* inc_ptr,
                                                          const int* inc_br, LossLaunch a) {
  __shared__ double red[4];
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
    double gr = 0.0, gi = 0.0;  // torch gradient dL/dRe + j dL/dIm = 2 sum conj(coef) I_f
    for (int q = inc_ptr[i]; q < inc_ptr[i + 1]; ++q) {
      const int k = inc_br[q];
      const int f = ext[net.br_f[k]], t = ext[net.br_t[k]];
      const double ysr = net.br_ys_re[k], ysi = net.br_ys_im[k], hb = 0.5 * net.br_b[k];
      const double vfr = v[2 * f], vfi = v[2 * f + 1], vtr = v[2 * t], vti = v[2 * t + 1];
      const double ir = ysr * vfr - (ysi + hb) * vfi - (ysr * vtr - ysi * vti);
      const double ii = ysr * vfi + (ysi + hb) * vfr - (ysr * vti + ysi * vtr);
      // coefficient of V_i in I_f: yff = ys + j b/2 at the from end, -ys at the to end
      double cr, ci;
      if (net.br_f[k] == i) {
        cr = ysr;
        ci = ysi + hb;
      } else {
        cr = -ysr;
        ci = -ysi;
      }
      // 2 conj(c) I
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
  hipLaunchKernelGGL(branch_loss_kernel, dim3(a.batch), dim3(256), 0, s, net.view<double>(),
                     net.inc_ptr.as<int>(), net.inc_br.as<int>(), a);
  PFX_HIP(hipGetLastError());
}

}  // namespace pfx
