// Batched Newton-Raphson power flow for meshed grids (Sec. II-A), one
// workgroup per scenario, and its adjoint.
//
// A workgroup owns one scenario for its whole solve.  Thread t owns internal
// buses i = t + k BLOCK (k < KB) and, for each, both Newton-state entries of
// that bus (angle and magnitude; see tx.hpp): vectors of the Newton space live
// in registers as w[k] (angle of bus slot k) and w[KB + k] (magnitude), and in
// HBM as two planes of nbp entries, so every streaming access is coalesced and
// per-scenario dot products are workgroup reductions.  No grid-wide
// synchronisation is ever needed.  Per-scenario data:
//   * LDS (about 40 KB at 2000 buses in FP64, so four workgroups share a CU):
//     the vector being gathered (V for Ybus V, dV for the Jacobian-vector
//     product, the preconditioner's right-hand sides), reduction partials, the
//     packed Hessenberg matrix and the Givens rotations;
//   * HBM (scenario-major workspace): theta, |V|, 1/|V|, V, I (the last three
//     as FP32 copies when the inner solve runs in FP32), P, Q, F, the Newton
//     step and the Krylov basis.
// Network data (sliced Ybus, G, the explicit factors of B' and B'') is shared
// by all workgroups and read through the caches; it is never written during a
// launch, so it is read through the constant address space.
//
// Steps per Newton iteration (eqs. (1)-(3), (7)-(9)):
//   mismatch  V = |V| e^{j theta}, I = Ybus V, S = V conj(I),
//             F = [Re S - P on Theta ; Im S - Q on Q], max |F|
//   GMRES     left-preconditioned restarted GMRES on J dx = -F with
//             Jacobian-vector products dS = dV conj(I) + V conj(Ybus dV),
//             dV = V (j dtheta + d|V| / |V|), the preconditioner applied by the
//             forward block substitution of eqs. (8)-(9) with explicit factor
//             passes, classical Gram-Schmidt with a second pass when the first
//             cancels all but 1/64 of the norm, Givens rotations on the
//             Hessenberg matrix
//   update    theta += dx_theta, |V| += dx_|V|   (FP64)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "device_ops.hpp"
#include "tx.hpp"

namespace pfx {

namespace {

template <int BLOCK>
__device__ __forceinline__ unsigned row(int k) {
  return threadIdx.x + (unsigned)k * BLOCK;
}

struct NrLayout {
  int xs, tmp, red, redn, H, cs, sn, gres, gfin, y, total;
};

__host__ __device__ inline int align16(int x) { return (x + 15) & ~15; }

// Column j of the packed Hessenberg matrix holds rows 0..j at offset j(j+1)/2.
__host__ __device__ inline int hcol(int j) { return j * (j + 1) / 2; }

__host__ __device__ inline NrLayout nr_layout(int nbp, int nth, int npq, int kmax, int R, int NW, int ts) {
  NrLayout L;
  int o = 0;
  int xs_bytes = 2 * nbp * 8;                          // V (FP64 pairs) in the mismatch
  if (2 * nbp * ts > xs_bytes) xs_bytes = 2 * nbp * ts;  // dV pairs in the Jacobian-vector product
  // the preconditioner's two right-hand sides and pass buffers: [0, 2 nth) and [nth, nth + npq)
  if (2 * nth * ts > xs_bytes) xs_bytes = 2 * nth * ts;
  if ((nth + npq) * ts > xs_bytes) xs_bytes = (nth + npq) * ts;
  L.xs = o;
  o += align16(xs_bytes);
  // Reduction partials, double-buffered.  The preconditioner's dense-core
  // right-hand side lives there too when it fits: no partial is pending while
  // the preconditioner runs (each phase in between ends with a barrier).
  const int red_bytes = 2 * (R + 2) * NW * 8;
  L.red = o;  o += align16(red_bytes);
  const int tmp_bytes = ((kmax > 0 ? kmax : 1) + 3) / 4 * 4 * ts;   // whole packs of the dense core
  if (tmp_bytes <= red_bytes) {
    L.tmp = L.red;
  } else {
    L.tmp = o;
    o += align16(tmp_bytes);
  }
  L.redn = o; o += align16(NW * 8);   // the norm reduction after the projection
  L.H = o;    o += align16(hcol(R) * ts);
  L.cs = o;   o += align16(R * ts);
  L.sn = o;   o += align16(R * ts);
  L.gres = o; o += align16((R + 1) * ts);
  L.gfin = o; o += align16(R * ts);
  L.y = o;    o += align16(R * ts);
  L.total = o;
  return L;
}

template <typename T>
struct Smem {
  T* xs;
  double2* vs;
  T* tmp;
  T* red;
  double* redd;
  T* redn;
  T* H;
  T* cs;
  T* sn;
  T* gres;
  T* gfin;
  T* yv;
};

template <typename T>
__device__ Smem<T> carve(unsigned char* smem, const NrLayout& L) {
  Smem<T> s;
  s.xs = reinterpret_cast<T*>(smem + L.xs);
  s.vs = reinterpret_cast<double2*>(smem + L.xs);
  s.tmp = reinterpret_cast<T*>(smem + L.tmp);
  s.red = reinterpret_cast<T*>(smem + L.red);
  s.redd = reinterpret_cast<double*>(smem + L.red);
  s.redn = reinterpret_cast<T*>(smem + L.redn);
  s.H = reinterpret_cast<T*>(smem + L.H);
  s.cs = reinterpret_cast<T*>(smem + L.cs);
  s.sn = reinterpret_cast<T*>(smem + L.sn);
  s.gres = reinterpret_cast<T*>(smem + L.gres);
  s.gfin = reinterpret_cast<T*>(smem + L.gfin);
  s.yv = reinterpret_cast<T*>(smem + L.y);
  return s;
}

// Raw buffer access to per-scenario memory: a buffer resource holds the base
// address (scalar registers), each lane supplies a 32-bit byte offset and the
// array/slot offset is a uniform (usually constant) scalar offset.  One lane
// offset then serves every array and every bus slot, so addresses take no
// vector registers beyond it.
struct Buf {
  __amdgpu_buffer_rsrc_t r;
};

__device__ __forceinline__ Buf make_buf(const void* base) {
  return Buf{__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, 0x7fffffff, 0x00020000)};
}

// Cache policy bits of the per-scenario streams (workspace and Krylov basis);
// 0 is the default policy.
constexpr int WS_POLICY = 0;
constexpr int BASIS_POLICY = 0;

template <typename T, int CP = 0>
__device__ __forceinline__ T bld(const Buf& b, unsigned voff, unsigned soff) {
  if constexpr (sizeof(T) == 8) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(b.r, (int)voff, (int)soff, CP);
    T d;
    __builtin_memcpy(&d, &v, 8);
    return d;
  } else {
    const auto v = __builtin_amdgcn_raw_buffer_load_b32(b.r, (int)voff, (int)soff, CP);
    T f;
    __builtin_memcpy(&f, &v, 4);
    return f;
  }
}

template <int CP = 0>
__device__ __forceinline__ void bst(const Buf& b, double x, unsigned voff, unsigned soff) {
  decltype(__builtin_amdgcn_raw_buffer_load_b64(b.r, 0, 0, 0)) v;
  __builtin_memcpy(&v, &x, 8);
  __builtin_amdgcn_raw_buffer_store_b64(v, b.r, (int)voff, (int)soff, CP);
}
template <int CP = 0>
__device__ __forceinline__ void bst(const Buf& b, float x, unsigned voff, unsigned soff) {
  decltype(__builtin_amdgcn_raw_buffer_load_b32(b.r, 0, 0, 0)) v;
  __builtin_memcpy(&v, &x, 4);
  __builtin_amdgcn_raw_buffer_store_b32(v, b.r, (int)voff, (int)soff, CP);
}

// One scenario's FP64 workspace: 13 planes of NBP = KB BLOCK doubles.  Plane
// F and DX span two planes each (angle plane, then magnitude plane).  With an
// even slot count a thread's slots 2j and 2j + 1 of a plane are adjacent
// (slot k of thread t at (k / G) G BLOCK + G t + k % G, G = 2), so that the
// pair is read or written with one 16-byte access.
enum WsPlane { TH = 0, VM, IVM, VRE, VIM, IRE, IIM, PIN, QIN, FP = 9, DXP = 11, WS_PLANES = 13 };

template <int BLOCK, int KB>
struct Ws {
  static constexpr unsigned NBP = (unsigned)KB * BLOCK;
  static constexpr int G = KB % 2 == 0 ? 2 : 1;
  Buf b;
  static __device__ __forceinline__ unsigned vo() { return threadIdx.x * (8u * G); }
  static __device__ __forceinline__ unsigned so(int a, int k) {
    return (unsigned)(a * (int)NBP + (k / G) * (G * BLOCK) + k % G) * 8u;
  }
  // plane a, bus slot k (k < 2 KB for the two-plane vectors F and DX)
  __device__ __forceinline__ double ld(int a, int k) const { return bld<double, WS_POLICY>(b, vo(), so(a, k)); }
  __device__ __forceinline__ void st(int a, int k, double v) const { bst<WS_POLICY>(b, v, vo(), so(a, k)); }
  // x[k] = slot k of plane a for k < N (N = KB, or 2 KB for F and DX), in pairs
  template <int N, typename T>
  __device__ __forceinline__ void ld_all(int a, T (&x)[N]) const {
#pragma unroll
    for (int k = 0; k < N; k += G) {
      if constexpr (G == 2) {
        double d0, d1;
        ld2(a, k, d0, d1);
        x[k] = (T)d0;
        x[k + 1] = (T)d1;
      } else {
        x[k] = (T)ld(a, k);
      }
    }
  }
  template <int N>
  __device__ __forceinline__ void st_all(int a, const double (&x)[N]) const {
#pragma unroll
    for (int k = 0; k < N; k += G) {
      if constexpr (G == 2) st2(a, k, x[k], x[k + 1]);
      else st(a, k, x[k]);
    }
  }
  // slots k and k + 1 (k even)
  __device__ __forceinline__ void ld2(int a, int k, double& x0, double& x1) const {
    if constexpr (G == 2) {
      const auto v = __builtin_amdgcn_raw_buffer_load_b128(b.r, (int)vo(), (int)so(a, k), WS_POLICY);
      double d[2];
      __builtin_memcpy(d, &v, 16);
      x0 = d[0];
      x1 = d[1];
    } else {
      x0 = ld(a, k);
      x1 = ld(a, k + 1);
    }
  }
  // Stores stay 8 bytes wide: with 16-byte stores here (whose data registers
  // the next loads reuse at once) some scenarios of batches above one
  // workgroup per CU read back wrong values, run to run differently.
  __device__ __forceinline__ void st2(int a, int k, double x0, double x1) const {
    st(a, k, x0);
    st(a, k + 1, x1);
  }
  // The mismatch's V, I and 1/|V| as the inner solve reads them: FP64 planes,
  // or for an FP32 inner solve FP32 copies in the same planes (V and I as
  // (re, im) pairs in one 8-byte slot of the VRE and IRE planes, 1/|V| in the
  // first half of the IVM slot), which halves their bytes per product.
  template <typename T>
  __device__ __forceinline__ void put_vi(int k, double vr, double vi, double ivm) const {
    if constexpr (sizeof(T) == 4) {
      st(VRE, k, pack2(vr, vi));
      bst<WS_POLICY>(b, (float)ivm, vo(), so(IVM, k));
    } else {
      st(VRE, k, vr);
      st(VIM, k, vi);
      st(IVM, k, ivm);
    }
  }
  template <typename T>
  __device__ __forceinline__ void put_i(int k, double ir, double ii) const {
    if constexpr (sizeof(T) == 4) {
      st(IRE, k, pack2(ir, ii));
    } else {
      st(IRE, k, ir);
      st(IIM, k, ii);
    }
  }
  template <typename T>
  __device__ __forceinline__ void get_v(int k, T& re, T& im) const {
    if constexpr (sizeof(T) == 4) {
      unpack2(ld(VRE, k), re, im);
    } else {
      re = ld(VRE, k);
      im = ld(VIM, k);
    }
  }
  template <typename T>
  __device__ __forceinline__ void get_i(int k, T& re, T& im) const {
    if constexpr (sizeof(T) == 4) {
      unpack2(ld(IRE, k), re, im);
    } else {
      re = ld(IRE, k);
      im = ld(IIM, k);
    }
  }
  template <typename T>
  __device__ __forceinline__ T get_ivm(int k) const {
    if constexpr (sizeof(T) == 4) {
      return bld<float, WS_POLICY>(b, vo(), so(IVM, k));
    } else {
      return ld(IVM, k);
    }
  }
  // The same for the slot pair k, k + 1 (k even)
  template <typename T>
  __device__ __forceinline__ void get_v2(int k, T (&re)[2], T (&im)[2]) const {
    if constexpr (sizeof(T) == 4) {
      double d0, d1;
      ld2(VRE, k, d0, d1);
      unpack2(d0, re[0], im[0]);
      unpack2(d1, re[1], im[1]);
    } else {
      ld2(VRE, k, re[0], re[1]);
      ld2(VIM, k, im[0], im[1]);
    }
  }
  template <typename T>
  __device__ __forceinline__ void get_i2(int k, T (&re)[2], T (&im)[2]) const {
    if constexpr (sizeof(T) == 4) {
      double d0, d1;
      ld2(IRE, k, d0, d1);
      unpack2(d0, re[0], im[0]);
      unpack2(d1, re[1], im[1]);
    } else {
      ld2(IRE, k, re[0], re[1]);
      ld2(IIM, k, im[0], im[1]);
    }
  }
  template <typename T>
  __device__ __forceinline__ void get_ivm2(int k, T (&iv)[2]) const {
    double d0, d1;
    ld2(IVM, k, d0, d1);
    if constexpr (sizeof(T) == 4) {
      float f0[2], f1[2];
      __builtin_memcpy(f0, &d0, 8);
      __builtin_memcpy(f1, &d1, 8);
      iv[0] = f0[0];
      iv[1] = f1[0];
    } else {
      iv[0] = d0;
      iv[1] = d1;
    }
  }

 private:
  static __device__ __forceinline__ double pack2(double x, double y) {
    const float f[2] = {(float)x, (float)y};
    double d;
    __builtin_memcpy(&d, f, 8);
    return d;
  }
  template <typename T>
  static __device__ __forceinline__ void unpack2(double d, T& x, T& y) {
    float f[2];
    __builtin_memcpy(f, &d, 8);
    x = f[0];
    y = f[1];
  }
};

// The Krylov basis of one scenario: vectors of MP = 2 NBP entries of T.  A
// thread's slots are stored in runs of G consecutive entries (G slots of 16
// bytes in all where the slot count allows), so that the compiler reads and
// writes a run with one wide access: slot k of thread t sits at
// (k / G) G BLOCK + G t + k % G.
template <typename T, int BLOCK, int KB>
struct Basis {
  static constexpr unsigned MP = 2u * KB * BLOCK;
  static constexpr int G = (16 / (int)sizeof(T) <= 2 * KB && (2 * KB) % (16 / (int)sizeof(T)) == 0)
                               ? 16 / (int)sizeof(T) : 2;
  Buf b;
  static __device__ __forceinline__ unsigned off(int i, int k) {
    return ((unsigned)i * MP + (unsigned)(k / G) * (G * BLOCK) + (unsigned)(k % G)) * (unsigned)sizeof(T);
  }
  // run g (slots g G .. g G + G - 1) of vector i: one load or store of G sizeof(T) bytes
  __device__ __forceinline__ void ldg(int i, int g, T* e) const {
    const unsigned vo = threadIdx.x * (unsigned)(G * sizeof(T)), so = off(i, g * G);
    if constexpr (G * sizeof(T) == 16) {
      const auto v = __builtin_amdgcn_raw_buffer_load_b128(b.r, (int)vo, (int)so, BASIS_POLICY);
      __builtin_memcpy(e, &v, 16);
    } else {
      const auto v = __builtin_amdgcn_raw_buffer_load_b64(b.r, (int)vo, (int)so, BASIS_POLICY);
      __builtin_memcpy(e, &v, 8);
    }
  }
  __device__ __forceinline__ void stg(int i, int g, const T* e) const {
    const unsigned vo = threadIdx.x * (unsigned)(G * sizeof(T)), so = off(i, g * G);
    if constexpr (G * sizeof(T) == 16) {
      decltype(__builtin_amdgcn_raw_buffer_load_b128(b.r, 0, 0, 0)) v;
      __builtin_memcpy(&v, e, 16);
      __builtin_amdgcn_raw_buffer_store_b128(v, b.r, (int)vo, (int)so, BASIS_POLICY);
    } else {
      decltype(__builtin_amdgcn_raw_buffer_load_b64(b.r, 0, 0, 0)) v;
      __builtin_memcpy(&v, e, 8);
      __builtin_amdgcn_raw_buffer_store_b64(v, b.r, (int)vo, (int)so, BASIS_POLICY);
    }
  }
};

// One group of four entries of a packed sliced layout (group index g) into
// v[0..3] and c[0..3]: one 8-byte load of the columns and sizeof(V) / 4
// 16-byte loads of the values.
template <typename V>
__device__ __forceinline__ void pgroup(const PSell<V>& a, unsigned g, V* v, int* c) {
  const int2 cc = cld(reinterpret_cast<const int2*>(a.col), g);
  c[0] = cc.x & 0xffff;
  c[1] = (int)((unsigned)cc.x >> 16);
  c[2] = cc.y & 0xffff;
  c[3] = (int)((unsigned)cc.y >> 16);
  constexpr int NL = (int)sizeof(V) / 4;
#pragma unroll
  for (int u = 0; u < NL; ++u) {
    const int4 q = cld(reinterpret_cast<const int4*>(a.val), (unsigned)NL * g + u);
    __builtin_memcpy(reinterpret_cast<char*>(v) + 16 * u, &q, 16);
  }
}

// One row (slice s, this lane) of a packed layout, a group per round.
template <typename V, typename Body>
__device__ __forceinline__ void psell_row(const PSell<V>& a, int s, Body&& body) {
  const int lane = lane_id();
  const int o = cld(a.off, (unsigned)s);
  const int wd = cld(a.width, (unsigned)s);
  for (int p = 0; p < wd; ++p) {
    V v[4];
    int c[4];
    pgroup(a, (unsigned)(o + p * WAVE + lane), v, c);
#pragma unroll
    for (int u = 0; u < 4; ++u) body(v[u], c[u]);
  }
}

// Rows by bus slot of a packed layout: the thread's bus slots k < KB are rows
// of slices k NW + wave.  body(k, val, col) accumulates one entry of slot k;
// after a slot's row, done(k) runs.
template <int KB, int NW, typename V, typename Body, typename Done>
__device__ __forceinline__ void psell_slots(const PSell<V>& a, Body&& body, Done&& done) {
  const int wv = wave_id();
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    psell_row(a, k * NW + wv, [&](V v, int c) { body(k, v, c); });
    done(k);
  }
}

// dst[r] = sum over row r of val * x[col] for the rows of a by-length packed
// layout (rid gives each lane's row, -1 for padding); rows in rounds of two
// groups (eight entries), then one group.
template <int KB, int NW, typename T>
__device__ __forceinline__ void sell_slots_store(const PSell<T>& a, const int* rid, const T* x, T* dst) {
  const int wv = wave_id(), lane = lane_id();
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    const unsigned sl = (unsigned)(k * NW + wv);
    const int o = cld(a.off, sl);
    const int wd = cld(a.width, sl);
    const int r = cld(rid, sl * WAVE + lane);
    T acc = 0;
    int p = 0;
    for (; p + 2 <= wd; p += 2) {
      T v[8];
      int c[8];
      pgroup(a, (unsigned)(o + p * WAVE + lane), v, c);
      pgroup(a, (unsigned)(o + (p + 1) * WAVE + lane), v + 4, c + 4);
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += v[u] * x[c[u]];
    }
    if (p < wd) {
      T v[4];
      int c[4];
      pgroup(a, (unsigned)(o + p * WAVE + lane), v, c);
#pragma unroll
      for (int u = 0; u < 4; ++u) acc += v[u] * x[c[u]];
    }
    if (r >= 0) dst[r] = acc;
  }
}

// acc[k] = sum over slot k's row of val * x[col] for a packed layout by bus
// slot (slices k NW + wave); rows in rounds of two groups, then one group.
template <int KB, int NW, typename T>
__device__ __forceinline__ void psell_slots_dot(const PSell<T>& a, const T* x, T (&acc)[KB]) {
  const int wv = wave_id(), lane = lane_id();
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    const unsigned sl = (unsigned)(k * NW + wv);
    const int o = cld(a.off, sl);
    const int wd = cld(a.width, sl);
    T s = 0;
    int p = 0;
    for (; p + 2 <= wd; p += 2) {
      T v[8];
      int c[8];
      pgroup(a, (unsigned)(o + p * WAVE + lane), v, c);
      pgroup(a, (unsigned)(o + (p + 1) * WAVE + lane), v + 4, c + 4);
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u] * x[c[u]];
    }
    if (p < wd) {
      T v[4];
      int c[4];
      pgroup(a, (unsigned)(o + p * WAVE + lane), v, c);
#pragma unroll
      for (int u = 0; u < 4; ++u) s += v[u] * x[c[u]];
    }
    acc[k] = s;
    settle(acc[k]);
  }
}

// out[OFF + k] = (A^-1 x)_i for the bus slots i = t + k BLOCK (zero past N), by
// the explicit factor passes E1 (rows into `aux` / the core right-hand side
// into `tmp`), E2 (dense core into aux past c), E3 (rows in matrix order, read
// from aux).  x holds the right-hand side in matrix order; aux (N entries)
// must not overlap it.  x is read only before the first barrier.  Two
// barriers (one when the core is empty); the caller places one before aux or
// tmp is written again.  A factor applied directly (f.direct) reads x
// throughout and has no barrier: the caller places one before x is written.
// With TO_LDS (not for a direct factor) E3 takes the by-length layout and
// stores x_i to dst[i] (i < N) instead of filling out; dst may be x itself,
// since x is no longer read by then.
template <typename T, int BLOCK, int KB, int OFF, int K, bool TO_LDS = false>
__device__ void efac_apply(const EfDev<T>& f, const T* x, T* aux, T* tmp, T (&out)[K], T* dst = nullptr) {
  constexpr int NW = BLOCK / WAVE;
  if (f.direct) {  // one sliced pass over A^-1 itself; no barrier, x read throughout
    T acc[KB];
    psell_slots_dot<KB, NW>(f.inv, x, acc);
#pragma unroll
    for (int k = 0; k < KB; ++k) out[OFF + k] = acc[k];
    return;
  }
  const int lane = lane_id(), wv = wave_id();
  // (kept rolled: the loop indexes no register array, and its body is large)
  const int nq = f.e1_nq;
#pragma unroll 1
  for (int q = 0; q < nq; ++q) {
    // (group offset, width in groups, first row) of this wave's q-th slice; width 0 past its list
    const int4 t = cld(reinterpret_cast<const int4*>(f.e1_wave), (unsigned)(wv * nq + q));
    if (t.y > 0) {
      const int r = cld(f.e1_row, (unsigned)(t.z + lane));
      T acc = 0;
      int p = 0;
      for (; p + 2 <= t.y; p += 2) {  // two groups (eight entries) in flight per round while they last
        T v[8];
        int c[8];
        pgroup(f.e1, (unsigned)(t.x + p * WAVE + lane), v, c);
        pgroup(f.e1, (unsigned)(t.x + (p + 1) * WAVE + lane), v + 4, c + 4);
#pragma unroll
        for (int u = 0; u < 8; ++u) acc += v[u] * x[c[u]];
      }
      if (p < t.y) {
        T v[4];
        int c[4];
        pgroup(f.e1, (unsigned)(t.x + p * WAVE + lane), v, c);
#pragma unroll
        for (int u = 0; u < 4; ++u) acc += v[u] * x[c[u]];
      }
      if (r >= f.c) tmp[r - f.c] = acc;
      else if (r >= 0) aux[r] = acc;
    }
  }
  {  // the dense core reads whole packs: zero the core right-hand side past k
    constexpr int P = 16 / (int)sizeof(T);
    const int pad = (f.k + P - 1) / P * P - f.k;
    if ((int)threadIdx.x < pad) tmp[f.k + threadIdx.x] = 0;
  }
  __syncthreads();
  // S^-1 is stored in packs of P = 16 / sizeof(T) consecutive columns per row
  // ([l / P][i][P], zero-padded), so each lane reads P entries with one
  // 16-byte load.
  constexpr int P = 16 / (int)sizeof(T);
  const int kp = (f.k + P - 1) / P;
  for (int i = threadIdx.x; i < f.k; i += BLOCK) {
    T acc[4] = {0, 0, 0, 0};
    int lp = 0;
    for (; lp + 7 < kp; lp += 8) {
      int4 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = cld(reinterpret_cast<const int4*>(f.sinv), (unsigned)((lp + u) * f.k + i));
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        T e[P];
        __builtin_memcpy(e, &v[u], 16);
#pragma unroll
        for (int q = 0; q < P; ++q) acc[q & 3] += e[q] * tmp[(lp + u) * P + q];
      }
    }
    for (; lp < kp; ++lp) {
      const int4 v = cld(reinterpret_cast<const int4*>(f.sinv), (unsigned)(lp * f.k + i));
      T e[P];
      __builtin_memcpy(e, &v, 16);
#pragma unroll
      for (int q = 0; q < P; ++q) acc[q & 3] += e[q] * tmp[lp * P + q];
    }
    aux[f.c + i] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  }
  if (f.k > 0) __syncthreads();  // with no core, E3 reads only what E1 wrote
  if constexpr (TO_LDS) {
    sell_slots_store<KB, NW>(f.e3s, f.e3s_row, aux, dst);
    return;
  }
  T acc[KB];
  psell_slots_dot<KB, NW>(f.e3, aux, acc);
#pragma unroll
  for (int k = 0; k < KB; ++k) out[OFF + k] = acc[k];
}

// z = M^-1 w for the left preconditioner of eq. (7), by the forward block
// substitution of eqs. (8)-(9):
//   z_Theta = (B' + eps I)^-1 diag(|V_Theta|)^-1 w_Theta
//   z_Q     = (B'' + eps I)^-1 diag(|V_Q|)^-1 (w_Q - G z_Theta)
// LDS use: the B' right-hand side at [0, nth) with its passes at [nth, 2 nth);
// z_Theta at [0, nth) (the B' factor's E3 pass stores it there directly,
// and each thread reads its own entries back); the B'' right-hand side at
// [nth, nth + npq) with its passes at [0, npq).  The caller guarantees that
// no thread still reads the LDS vector area.
template <typename T, int BLOCK, int KB>
__device__ void precond(const TxDev<T>* netp, const Ws<BLOCK, KB>& ws, T (&w)[2 * KB], const Smem<T>& s) {
  constexpr int NW = BLOCK / WAVE;
  const TxDev<T> net = load_desc(netp);
  const unsigned nth = net.nth, npq = net.npq;
  T* X = s.xs;
  T* Y = s.xs + nth;
  constexpr int G = Ws<BLOCK, KB>::G;
#pragma unroll
  for (int k = 0; k < KB; k += G) {
    T iv[2];
    if constexpr (G == 2) ws.template get_ivm2<T>(k, iv);
    else iv[0] = ws.template get_ivm<T>(k);
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const unsigned i = row<BLOCK>(k + u);
      const T v = w[k + u] * iv[u];
      if (i < nth) X[i] = v;
    }
  }
  __syncthreads();
  if (net.bp.direct) {
    efac_apply<T, BLOCK, KB, 0>(net.bp, X, Y, s.tmp, w);
    if (npq > 0) {
      // the direct pass read X throughout; the barrier after the stores also
      // orders its reads of Y before Y is written again
      __syncthreads();
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        const unsigned i = row<BLOCK>(k);
        if (i < nth) X[i] = w[k];
      }
      __syncthreads();
    }
  } else {
    // X was last read before the first barrier of the B' passes, so their
    // E3 pass stores z_Theta over it; the barrier also orders the passes'
    // reads of Y before Y is written again.
    efac_apply<T, BLOCK, KB, 0, 2 * KB, true>(net.bp, X, Y, s.tmp, w, X);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const unsigned i = row<BLOCK>(k);
      w[k] = i < nth ? X[i] : (T)0;
    }
  }
  if (npq > 0) {
    const TxDev<T> nt = load_desc(netp);
    // 1/|V| requested before the G pass, so its latency overlaps the pass
    T iv[KB];
#pragma unroll
    for (int k = 0; k < KB; k += G) {
      if constexpr (G == 2) {
        T t[2];
        ws.template get_ivm2<T>(k, t);
        iv[k] = t[0];
        iv[k + 1] = t[1];
      } else {
        iv[k] = ws.template get_ivm<T>(k);
      }
    }
    T gz[KB];
    psell_slots_dot<KB, NW>(nt.g, X, gz);
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const unsigned i = row<BLOCK>(k);
      const T t = (w[KB + k] - gz[k]) * iv[k];
      if (i < npq) Y[i] = t;
    }
    __syncthreads();
    efac_apply<T, BLOCK, KB, KB>(nt.bpp, Y, X, s.tmp, w);
  }
}

// w <- J w, the Jacobian of the mismatch at the current V (with I = Ybus V).
// yv: the scenario's own Ybus values (layout of net.yT), or null for the
// network's.  Ends with a barrier.
template <typename T, int BLOCK, int KB>
__device__ void jvp(const TxDev<T>* netp, const Ws<BLOCK, KB>& ws, T (&w)[2 * KB], T* lds,
                    const typename Vec2<T>::type* yv) {
  using T2 = typename Vec2<T>::type;
  TxDev<T> net = load_desc(netp);
  if (yv) net.yT.val = yv;
  constexpr int NW = BLOCK / WAVE;
  const unsigned nth = net.nth, npq = net.npq;
  T2* dv = reinterpret_cast<T2*>(lds);
  // dV_i = V_i (j p_theta + p_|V| / |V|).  The input w is dead after this
  // loop, so the own buses' V stays in its registers for the second phase.
  constexpr int G = Ws<BLOCK, KB>::G;
  T vre[KB], vim[KB];
#pragma unroll
  for (int k = 0; k < KB; k += G) {
    T iv[2];
    if constexpr (G == 2) {
      ws.template get_ivm2<T>(k, iv);
      T re[2], im[2];
      ws.template get_v2<T>(k, re, im);
      vre[k] = re[0];
      vre[k + 1] = re[1];
      vim[k] = im[0];
      vim[k + 1] = im[1];
    } else {
      iv[0] = ws.template get_ivm<T>(k);
      ws.template get_v<T>(k, vre[k], vim[k]);
    }
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const unsigned i = row<BLOCK>(k + u);
      const T a = w[KB + k + u] * iv[u];
      T2 d;
      d.x = vre[k + u] * a - vim[k + u] * w[k + u];
      d.y = vim[k + u] * a + vre[k + u] * w[k + u];
      dv[i] = d;
    }
  }
  __syncthreads();
  // The own buses' I is fetched one slot pair ahead, so its HBM latency
  // overlaps the previous slots' rows.
  const int wv = wave_id();
  T cIr[2], cIi[2], nIr[2], nIi[2];
  if constexpr (G == 2) ws.template get_i2<T>(0, nIr, nIi);
  else ws.template get_i<T>(0, nIr[0], nIi[0]);
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    if (k % G == 0) {
      cIr[0] = nIr[0];
      cIi[0] = nIi[0];
      cIr[1] = nIr[1];
      cIi[1] = nIi[1];
      if (k + G < KB) {
        if constexpr (G == 2) ws.template get_i2<T>(k + G, nIr, nIi);
        else ws.template get_i<T>(k + G, nIr[0], nIi[0]);
      }
    }
    const T Ir = cIr[k % G], Ii = cIi[k % G], vr = vre[k], vi = vim[k];
    T dIr = 0, dIi = 0;
    psell_row(net.yT, k * NW + wv, [&](T2 y, int c) {
      const T2 d = dv[c];
      dIr += y.x * d.x - y.y * d.y;
      dIi += y.x * d.y + y.y * d.x;
    });
    const unsigned i = row<BLOCK>(k);
    const T2 d = dv[i];
    // dS = dV conj(I) + V conj(dI): real part on Theta, imaginary part on Q
    w[k] = i < nth ? d.x * Ir + d.y * Ii + vr * dIr + vi * dIi : (T)0;
    w[KB + k] = i < npq ? d.y * Ir - d.x * Ii + vi * dIr - vr * dIi : (T)0;
    settle(w[k]);
    settle(w[KB + k]);
  }
  __syncthreads();
}

// Writes part[i NW + wave] = the wave's share of <basis_i, w> for i < nv and
// part[nv NW + wave] = the wave's share of ss; ends with a barrier.
template <typename T, int BLOCK, int KB>
__device__ void multi_dot(const Basis<T, BLOCK, KB>& basis, int nv, const T (&w)[2 * KB], T ss, T* part) {
  constexpr int NW = BLOCK / WAVE;
  const int lane = lane_id(), wid = wave_id();
  int i = 0;
  constexpr int G = Basis<T, BLOCK, KB>::G;
  for (; i + 1 < nv; i += 2) {  // two vectors per round: twice the loads in flight
    T a0 = 0, a1 = 0;
#pragma unroll
    for (int g = 0; g < 2 * KB / G; ++g) {
      T e0[G], e1[G];
      basis.ldg(i, g, e0);
      basis.ldg(i + 1, g, e1);
#pragma unroll
      for (int q = 0; q < G; ++q) {
        a0 += e0[q] * w[g * G + q];
        a1 += e1[q] * w[g * G + q];
      }
    }
    a0 = wave_total(a0);
    a1 = wave_total(a1);
    if (lane == 0) {
      part[i * NW + wid] = a0;
      part[(i + 1) * NW + wid] = a1;
    }
  }
  if (i < nv) {
    T a0 = 0;
#pragma unroll
    for (int g = 0; g < 2 * KB / G; ++g) {
      T e0[G];
      basis.ldg(i, g, e0);
#pragma unroll
      for (int q = 0; q < G; ++q) a0 += e0[q] * w[g * G + q];
    }
    a0 = wave_total(a0);
    if (lane == 0) part[i * NW + wid] = a0;
  }
  ss = wave_total(ss);
  if (lane == 0) part[nv * NW + wid] = ss;
  __syncthreads();
}

template <typename T, int NW>
__device__ __forceinline__ T part_sum(const T* part, int i) {
  T s = 0;
#pragma unroll
  for (int u = 0; u < NW; ++u) s += part[i * NW + u];
  return s;
}

// w -= sum_i h_i basis_i with h_i from the partials; returns sum_i h_i^2.
template <typename T, int BLOCK, int KB>
__device__ T subtract_proj(const Basis<T, BLOCK, KB>& basis, int nv, T (&w)[2 * KB], const T* part) {
  constexpr int NW = BLOCK / WAVE;
  constexpr int G = Basis<T, BLOCK, KB>::G;
  T hh = 0;
  int i = 0;
  for (; i + 1 < nv; i += 2) {
    const T h0 = part_sum<T, NW>(part, i), h1 = part_sum<T, NW>(part, i + 1);
    hh += h0 * h0 + h1 * h1;
#pragma unroll
    for (int g = 0; g < 2 * KB / G; ++g) {
      T e0[G], e1[G];
      basis.ldg(i, g, e0);
      basis.ldg(i + 1, g, e1);
#pragma unroll
      for (int q = 0; q < G; ++q) w[g * G + q] -= h0 * e0[q] + h1 * e1[q];
    }
  }
  if (i < nv) {
    const T h0 = part_sum<T, NW>(part, i);
    hh += h0 * h0;
#pragma unroll
    for (int g = 0; g < 2 * KB / G; ++g) {
      T e0[G];
      basis.ldg(i, g, e0);
#pragma unroll
      for (int q = 0; q < G; ++q) w[g * G + q] -= h0 * e0[q];
    }
  }
  return hh;
}

// Mismatch at the current (theta, |V|): writes V, 1/|V|, I and F to the
// workspace and returns max |F| (NaN if any entry is NaN).  yv: the scenario's
// own Ybus values (layout of net.y64), or null.  Ends with a barrier.
template <typename T, int BLOCK, int KB>
__device__ double mismatch(const TxDev<T>* netp, const Ws<BLOCK, KB>& ws, double2* vs, double* part,
                           const double2* yv) {
  constexpr int NW = BLOCK / WAVE;
  TxDev<T> net = load_desc(netp);
  if (yv) net.y64.val = yv;
  const unsigned nth = net.nth, npq = net.npq;
  // every slot's angle and magnitude requested at once (in pairs), then one
  // slot at a time through sincos
  double th[KB], vmag[KB];
  ws.ld_all(TH, th);
  ws.ld_all(VM, vmag);
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    slot_fence();
    const unsigned i = row<BLOCK>(k);
    double sn, cs;
    sincos(th[k], &sn, &cs);
    const double vm = vmag[k];
    double2 v;
    v.x = vm * cs;
    v.y = vm * sn;
    ws.template put_vi<T>(k, v.x, v.y, 1.0 / vm);
    vs[i] = v;
  }
  __syncthreads();
  const int wv = wave_id();
  double fmax = 0.0;
  double pin[KB], qin[KB];
  ws.ld_all(PIN, pin);
  ws.ld_all(QIN, qin);
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    const double pk = pin[k], qk = qin[k];
    double Ir = 0.0, Ii = 0.0;
    psell_row(net.y64, k * NW + wv, [&](double2 y, int c) {
      const double2 v = vs[c];
      Ir += y.x * v.x - y.y * v.y;
      Ii += y.x * v.y + y.y * v.x;
    });
    const unsigned i = row<BLOCK>(k);
    const double2 v = vs[i];
    ws.template put_i<T>(k, Ir, Ii);
    const double ft = i < nth ? v.x * Ir + v.y * Ii - pk : 0.0;
    const double fv = i < npq ? v.y * Ir - v.x * Ii - qk : 0.0;
    ws.st(FP, k, ft);
    ws.st(FP, KB + k, fv);
    fmax = nanmax(fmax, nanmax(fabs(ft), fabs(fv)));
    settle(fmax);
  }
  return block_nanmax<BLOCK>(fmax, part);
}

// Algorithmic HBM bytes of one scenario (the byte model reported with the
// solve): with w = sizeof(T), per Jacobian-vector product 2 w m + 4 w n, per
// preconditioner application 2 w m + 8 n, per Gram-Schmidt pass of Arnoldi
// step j (against j + 1 vectors) (2 j + 3) w m, per cycle start 8 m + w m,
// per cycle end (k + 2) w m, per mismatch evaluation 32 n + 16 m and per
// Newton update 16 m.
struct ByteModel {
  double wm, m8, n8;
  // V and I (four reals per bus) read by a Jacobian-vector product: FP64, or
  // their FP32 copies for an FP32 inner solve
  double vi_n;
  // per-scenario Ybus entries read by a Jacobian-vector product and by a
  // mismatch evaluation (zero when the network's shared values are used)
  double yj = 0.0, ym = 0.0;
  __device__ double jvp() const { return 2 * wm + vi_n + yj; }
  __device__ double pre() const { return 2 * wm + n8; }
  __device__ double orth_pass(int j) const { return (2.0 * j + 3.0) * wm; }
  __device__ double mismatch() const { return 4 * n8 + 2 * m8 + ym; }
  __device__ double update() const { return 2 * m8; }
};

// Restarted GMRES with left preconditioning for A x = b from x = 0, where
// apply_a(w) overwrites w with A w and apply_m(w) with M^-1 w (both on the
// thread's own rows).  b is read from `rhs` (FP64, own rows); x accumulates in
// FP64 in `x` (own rows).  Stops when the Givens estimate of
// ||M^-1 (b - A x)|| reaches rtol ||M^-1 b||, after max_restarts cycles, or at
// a breakdown.  Returns the number of Arnoldi steps; *converged tells whether
// the tolerance was met.
//
// Orthogonalisation: one reduction gives <v_i, w> and ||w||^2 together;
// ||w'||^2 after the projection is their difference unless it cancels or the
// tolerance is tight (then a second reduction); a second classical
// Gram-Schmidt pass runs when the
// projection leaves less than 1/64 of the norm.  Every thread applies the Givens
// rotations to the new Hessenberg column itself (same data, same operations),
// so no barrier is needed after them; thread 0 alone stores H, the rotations
// and the rotated right-hand side for later steps.
template <typename T, int BLOCK, int KB, typename ApplyA, typename ApplyM>
__device__ int gmres_solve(ApplyA&& apply_a, ApplyM&& apply_m, const Ws<BLOCK, KB>& ws, int bpl, int xpl,
                           const Basis<T, BLOCK, KB>& basis, int R, int max_restarts, T rtol, const Smem<T>& s,
                           bool* converged, const ByteModel& bm, double* work) {
  constexpr int NW = BLOCK / WAVE;
  constexpr int K = 2 * KB;
  constexpr int G = Basis<T, BLOCK, KB>::G;
  const unsigned pstride = (unsigned)(R + 2) * NW;
  int par = 0;
  auto next_part = [&]() {
    T* p = s.red + par * pstride;
    par ^= 1;
    return p;
  };
  T w[K];
  T beta0 = 0;
  int total = 0;
  bool done = false;
  {
    double z[K];
#pragma unroll
    for (int k = 0; k < K; ++k) z[k] = 0.0;
    ws.st_all(xpl, z);
  }
  for (int cycle = 0; cycle < max_restarts && !done; ++cycle) {
    *work += (cycle > 0 ? bm.jvp() : 0.0) + bm.pre() + bm.m8 + bm.wm;
    int steps = 0;
    T res = 0;
    bool stop = false;
    // Step -1 starts the cycle (w = M^-1 (b - A x)); steps j >= 0 are Arnoldi
    // steps.  One call site for A and one for M^-1 keeps the loop's code
    // compact (they are inlined).
    for (int j = -1; j < R; ++j) {
      if (j < 0) ws.ld_all(cycle == 0 ? bpl : xpl, w);
      if (j >= 0 || cycle > 0) apply_a(w);
      if (j < 0 && cycle > 0) {
        T bv[K];
        ws.ld_all(bpl, bv);
#pragma unroll
        for (int k = 0; k < K; ++k) w[k] = bv[k] - w[k];
      }
      apply_m(w);
      if (j < 0) {
        T ss = 0;
#pragma unroll
        for (int k = 0; k < K; ++k) ss += w[k] * w[k];
        const T beta = sqrt(block_sum<T, BLOCK>(ss, next_part()));
        if (cycle == 0) beta0 = beta;
        if (!(beta > rtol * beta0) || beta == (T)0) {
          done = !(beta > rtol * beta0);
          stop = true;
          break;
        }
        const T ib = (T)1 / beta;
#pragma unroll
        for (int k = 0; k < K; ++k) w[k] *= ib;
#pragma unroll
        for (int g = 0; g < K / G; ++g) basis.stg(0, g, w + g * G);
        if (threadIdx.x == 0) s.gres[0] = beta;
        res = beta;
        continue;
      }
      T ss0 = 0;
#pragma unroll
      for (int k = 0; k < K; ++k) ss0 += w[k] * w[k];
      T* p1 = next_part();
      multi_dot<T, BLOCK, KB>(basis, j + 1, w, ss0, p1);
      const T hh1 = subtract_proj<T, BLOCK, KB>(basis, j + 1, w, p1);
      const T wn2 = part_sum<T, NW>(p1, j + 1);
      // ||w'||^2 = ||w||^2 - sum h_i^2, unless that difference has cancelled
      // below tau ||w||^2 (its relative error is then above eps / tau): then
      // by its own reduction.  The identity assumes an orthonormal basis; its
      // error grows with the basis's loss of orthogonality, which matters
      // only for tight tolerances (with it, the adjoint's 1e-10 solves took
      // 2.7 times the steps), so below rtol 1e-6 the norm is always reduced.
      // Every thread takes the same branch (the same partials, summed in the
      // same order, and the same rtol).
      T s1 = 0;
#pragma unroll
      for (int k = 0; k < K; ++k) s1 += w[k] * w[k];
      T nrm2 = wn2 - hh1;
      constexpr T tau = sizeof(T) == 8 ? (T)1e-4 : (T)1e-3;
      if (!(rtol >= (T)1e-6) || !(nrm2 >= tau * wn2)) nrm2 = block_sum<T, BLOCK>(s1, s.redn);
      // Second pass only when the projection removed all but 1/64 of the
      // norm: the first pass's rounding then leaves the new vector orthogonal
      // to about 64 ulp, far below the GMRES tolerance, and a pass is saved in
      // most steps.
      const bool again = nrm2 < (T)(1.0 / 4096.0) * wn2;
      T* p2 = p1;
      if (again) {
        p2 = next_part();
        multi_dot<T, BLOCK, KB>(basis, j + 1, w, s1, p2);
        const T hh2 = subtract_proj<T, BLOCK, KB>(basis, j + 1, w, p2);
        nrm2 = nrm2 - hh2;   // the second pass removes only a small remainder
      }
      *work += bm.jvp() + bm.pre() + (again ? 2 : 1) * bm.orth_pass(j);
      const T hn = sqrt(nrm2 > (T)0 ? nrm2 : (T)0);
      // Hessenberg column j: h_i (+ second-pass h_i), rotated by the previous Givens rotations
      T* Hj = s.H + hcol(j);
      T cur = part_sum<T, NW>(p1, 0) + (again ? part_sum<T, NW>(p2, 0) : (T)0);
      for (int i = 0; i < j; ++i) {
        const T nxt = part_sum<T, NW>(p1, i + 1) + (again ? part_sum<T, NW>(p2, i + 1) : (T)0);
        const T c = s.cs[i], sn = s.sn[i];
        const T a = c * cur + sn * nxt;
        cur = -sn * cur + c * nxt;
        if (threadIdx.x == 0) Hj[i] = a;
      }
      const T d = sqrt(cur * cur + hn * hn);
      const T c = d == (T)0 ? (T)1 : cur / d;
      const T sn = d == (T)0 ? (T)0 : hn / d;
      const T gj = s.gres[j];
      const T gnext = -sn * gj;
      if (threadIdx.x == 0) {
        Hj[j] = d;
        s.cs[j] = c;
        s.sn[j] = sn;
        s.gres[j + 1] = gnext;
        s.gfin[j] = c * gj;
      }
      res = fabs(gnext);
      steps = j + 1;
      if (!(res > rtol * beta0) || j == R - 1 || !(hn > (T)0)) break;
      const T ih = (T)1 / hn;
#pragma unroll
      for (int k = 0; k < K; ++k) w[k] *= ih;
#pragma unroll
      for (int g = 0; g < K / G; ++g) basis.stg(j + 1, g, w + g * G);
    }
    if (stop) break;
    total += steps;
    *work += (steps + 2) * bm.wm;
    // y = H^-1 g (upper triangular after the rotations)
    if (threadIdx.x == 0) {
      for (int i = steps - 1; i >= 0; --i) {
        T a = s.gfin[i];
        for (int l = i + 1; l < steps; ++l) a -= s.H[hcol(l) + i] * s.yv[l];
        const T d = s.H[hcol(i) + i];
        s.yv[i] = d != (T)0 ? a / d : (T)0;
      }
    }
    __syncthreads();
    // x += V y: the basis vector index outermost, so each vector's loads
    // for all bus slots are in flight together
    {
      double acc[K];
      ws.ld_all(xpl, acc);
      int i = 0;
      for (; i + 1 < steps; i += 2) {  // two vectors' loads in flight per round
        const double y0 = (double)s.yv[i], y1 = (double)s.yv[i + 1];
#pragma unroll
        for (int g = 0; g < K / G; ++g) {
          T e0[G], e1[G];
          basis.ldg(i, g, e0);
          basis.ldg(i + 1, g, e1);
#pragma unroll
          for (int q = 0; q < G; ++q) {
            acc[g * G + q] += y0 * (double)e0[q];
            acc[g * G + q] += y1 * (double)e1[q];
          }
        }
      }
      if (i < steps) {
        const double yi = (double)s.yv[i];
#pragma unroll
        for (int g = 0; g < K / G; ++g) {
          T e[G];
          basis.ldg(i, g, e);
#pragma unroll
          for (int q = 0; q < G; ++q) acc[g * G + q] += yi * (double)e[q];
        }
      }
      ws.st_all(xpl, acc);
    }
    done = !(res > rtol * beta0);
  }
  *converged = done;
  return total;
}

template <typename T, int BLOCK, int KB>
// Four waves per SIMD: with about 40 KB of LDS per scenario, four workgroups
// (four scenarios) share a CU; registers are capped to match.
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void nr_kernel(
    const TxDev<T>* __restrict__ netp, NRLaunch a) {
  constexpr int NW = BLOCK / WAVE;
  constexpr int K = 2 * KB;
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = a.slots ? a.slots[blockIdx.x] : (int)blockIdx.x;
  int n, npq, kmax;
  {
    const TxDev<T> net = load_desc(netp);
    n = net.n;
    npq = net.npq;
    kmax = net.bp.k > net.bpp.k ? net.bp.k : net.bpp.k;
  }
  NrSlotState* const sst = a.state ? a.state + b : nullptr;
  const int phase = sst ? sst->phase : 0;
  if (phase == 2) {  // finished in an earlier launch: nothing to do
    if (threadIdx.x == 0) a.step_done[blockIdx.x] = 1;
    return;
  }
  const int R = a.restart;
  const NrLayout L = nr_layout(KB * BLOCK, n - 1, npq, kmax, R, NW, (int)sizeof(T));
  const Smem<T> s = carve<T>(smem, L);

  const Ws<BLOCK, KB> ws{make_buf(a.ws_d + (int64_t)b * a.ws_d_stride)};
  const Basis<T, BLOCK, KB> basis{make_buf(reinterpret_cast<T*>(a.ws_basis) + (int64_t)b * a.ws_b_stride)};
  const Buf P = make_buf(a.p_inj + (int64_t)b * a.ld);
  const Buf Q = make_buf(a.q_inj + (int64_t)b * a.ld);
  const Buf VS = make_buf(a.vm_set + (int64_t)b * a.ld);

  // flat start: theta = 0, |V| = set-point at PV and slack, 1 at PQ buses;
  // scheduled injections in internal order (padding buses: |V| = 1, no injection)
  if (phase == 0) {
    const TxDev<T> net = load_desc(netp);
    // every slot's inputs gathered before any workspace store (the stores
    // would otherwise hold back the next slot's loads)
    double p[KB], q[KB], vs[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const unsigned i = row<BLOCK>(k);
      p[k] = 0.0;
      q[k] = 0.0;
      vs[k] = 1.0;
      if ((int)i < n) {
        const unsigned e = (unsigned)cld(net.int2ext, i) * 8u;
        p[k] = bld<double>(P, e, 0);
        q[k] = bld<double>(Q, e, 0);
        if ((int)i >= npq) vs[k] = bld<double>(VS, e, 0);
      }
    }
    double zero[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) zero[k] = 0.0;
    ws.st_all(TH, zero);
    ws.st_all(VM, vs);
    ws.st_all(PIN, p);
    ws.st_all(QIN, q);
  }

  using T2 = typename Vec2<T>::type;
  const double2* yv64 = a.yv64 ? a.yv64 + (int64_t)b * a.yv_stride : nullptr;
  const T2* yvT = a.yvT ? reinterpret_cast<const T2*>(a.yvT) + (int64_t)b * a.yv_stride : nullptr;
  auto apply_j = [&](T (&w)[K]) { jvp<T, BLOCK, KB>(netp, ws, w, s.xs, yvT); };
  auto apply_m = [&](T (&w)[K]) { precond<T, BLOCK, KB>(netp, ws, w, s); };

  int newton = 0, gtotal = 0;
  bool conv = false;
  double fnorm = 0.0;
  double work = 0.0;
  double fprev = 0.0, eta = 0.0;   // the previous step's |F| and forcing term
  int par = 0;
  // A resumed scenario's workspace already holds the mismatch of its
  // iterate (tested before it was saved), so it goes straight to the solve.
  bool resume = phase == 1;
  if (resume) {
    newton = sst->newton;
    gtotal = sst->gtotal;
    fnorm = sst->fnorm;
    work = sst->work;
    fprev = sst->fprev;
    eta = sst->eta;
  }
  int steps = 0;
  for (;;) {
    const TxDev<T> net = load_desc(netp);
    const ByteModel bm{(double)sizeof(T) * net.m, 8.0 * net.m, 8.0 * n, 4.0 * sizeof(T) * n,
                       2.0 * sizeof(T) * a.yv_nnz, 16.0 * a.yv_nnz};
    if (!resume) {
      fnorm = mismatch<T, BLOCK, KB>(netp, ws, s.vs, s.redd + par * NW, yv64);
      work += bm.mismatch();
      par ^= 1;
      if (!(fnorm <= a.diverge)) break;
      if (fnorm <= a.tol) {
        conv = true;
        break;
      }
      if (newton >= a.max_newton) break;
      if (sst && steps >= a.step_iters) {
        // out of this launch's steps: keep the state for the next launch
        if (threadIdx.x == 0) {
          sst->phase = 1;
          sst->newton = newton;
          sst->gtotal = gtotal;
          sst->fnorm = fnorm;
          sst->work = work;
          sst->fprev = fprev;
          sst->eta = eta;
          a.step_done[blockIdx.x] = 0;
        }
        return;
      }
    }
    resume = false;
    // Inexact Newton: the linear solve's relative tolerance.  Adaptive
    // (Eisenstat and Walker's choice 2): loose while far from the solution,
    // tightening with the square of the mismatch's decrease, but never
    // tighter than the fixed tolerance rtol nor than reaching tol from the
    // current mismatch requires.
    double rt = a.rtol;
    if (a.forcing) {
      double e = a.forcing_max;
      if (newton > 0) {
        const double q = fnorm / fprev;
        e = 0.9 * q * q;
        const double safe = 0.9 * eta * eta;
        if (safe > 0.1 && safe > e) e = safe;
        if (e > a.forcing_max) e = a.forcing_max;
      }
      const double floor = 0.1 * a.tol / fnorm;
      if (e < floor) e = floor;
      if (e < a.rtol) e = a.rtol;
      eta = e;
      rt = e;
    }
    fprev = fnorm;
    // right-hand side -F in place (own rows)
    {
      double f[K];
      ws.ld_all(FP, f);
#pragma unroll
      for (int k = 0; k < K; ++k) f[k] = -f[k];
      ws.st_all(FP, f);
    }
    bool lin_ok;
    gtotal += gmres_solve<T, BLOCK, KB>(apply_j, apply_m, ws, FP, DXP, basis, R, a.max_restarts, (T)rt, s,
                                        &lin_ok, bm, &work);
    // Newton update (eq. (3)), FP64, own buses
    {
      // every load before the first store (a store holds back later loads)
      double th[KB], vm[KB], dx[K];
      ws.ld_all(TH, th);
      ws.ld_all(VM, vm);
      ws.ld_all(DXP, dx);
#pragma unroll
      for (int k = 0; k < KB; ++k) {
        th[k] += dx[k];
        vm[k] += dx[KB + k];
      }
      ws.st_all(TH, th);
      ws.st_all(VM, vm);
    }
    work += bm.update();
    ++newton;
    ++steps;
  }

  const Buf vout = make_buf(a.v_out + 2 * (int64_t)b * a.ld);
  {
    const TxDev<T> net = load_desc(netp);
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const unsigned i = row<BLOCK>(k);
      if ((int)i < n) {
        const unsigned e = (unsigned)cld(net.int2ext, i) * 16u;
        // V of the last iterate, formed exactly as the last mismatch formed it
        double sn, cs;
        sincos(ws.ld(TH, k), &sn, &cs);
        const double vm = ws.ld(VM, k);
        bst(vout, vm * cs, e, 0);
        bst(vout, vm * sn, e, 8);
      }
    }
  }
  if (threadIdx.x == 0) {
    a.newton_iters[b] = newton;
    if (a.gmres_iters) a.gmres_iters[b] = gtotal;
    a.converged[b] = conv ? 1 : 0;
    if (a.final_mismatch) a.final_mismatch[b] = fnorm;
    if (a.work_bytes) a.work_bytes[b] = work;
    if (sst) {
      sst->phase = 2;
      a.step_done[blockIdx.x] = 1;
    }
  }
}

// ---------------------------------------------------------------------------
// Direct Newton step (FP64): per scenario, the Jacobian of eq. (4) is formed
// in the shared fill pattern (direct.hpp), factorised by LU without pivoting
// in the shared minimum-degree order and solved by the two triangular
// solves; one workgroup per scenario with the factor in LDS.  Both the
// factorisation (with the forward solve inside it) and the backward solve run
// one phase per level of the elimination tree, with the phase's targets
// (rows) spread over the workgroup.
//
// Entries of J for a Ybus entry (i, k), with a = V_i conj(Y_ik V_k) and
// c = V_i conj(I_i) (the bus power):  i != k: dS_i/dtheta_k = -j a,
// dS_i/d|V_k| = a / |V_k|;  i == k: dS_i/dtheta_i = j (c - a),
// dS_i/d|V_i| = (a + c) / |V_i|.  Theta rows take the real part, Q rows the
// imaginary part (kind = 2 row type + column type).
// Byte offset of the staged schedule tables in the direct kernel's LDS.
__host__ __device__ inline size_t direct_stage_offset(int nbp, int nw, const DirectDev& d) {
  return ((size_t)2 * nbp * 16 + (size_t)2 * nw * 8 + ((size_t)d.n_val + 2 * d.m) * 8 + 15) / 16 * 16;
}
__host__ __device__ inline size_t direct_stage_bytes(const DirectDev& d) {
  return (size_t)16 * (d.n_tg + d.n_ct + d.n_je) +
         (size_t)4 * ((d.m + 1) + d.n_s + d.m + (d.n_fph + 1) + (d.n_bph + 1));
}

// STAGE: the schedule tables (targets, contributions, J entries, S(k) and the
// level lists) are copied into LDS once per workgroup, so each phase reads
// them at LDS latency instead of an L2 round trip (when they fit).
// VG: the factor values live in device memory (a.ws_dval, per scenario)
// instead of LDS, for factors larger than the LDS can hold; the level
// barriers order their reads and writes within the workgroup as before.
template <int BLOCK, int KB, bool STAGE, bool VG>
__global__ __launch_bounds__(BLOCK) void nr_direct_kernel(const TxDev<double>* __restrict__ netp, DirectDev d,
                                                          NRLaunch a) {
  constexpr int NW = BLOCK / WAVE;
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = blockIdx.x, tid = threadIdx.x;
  int n, npq, nth;
  {
    const TxDev<double> net = load_desc(netp);
    n = net.n;
    npq = net.npq;
    nth = net.nth;
  }
  constexpr int NBP = KB * BLOCK;
  const int m = d.m, ns = d.n_s;
  double2* vs = reinterpret_cast<double2*>(smem);
  double2* is = vs + NBP;
  double* red = reinterpret_cast<double*>(is + NBP);
  double* rhs = red + 2 * NW + (VG ? 0 : d.n_val);
  double* xs = rhs + m;
  double* val = VG ? a.ws_dval + (int64_t)b * a.ws_dval_stride : red + 2 * NW;
  int4 *ltg = nullptr, *lct = nullptr, *lje = nullptr;
  int *lso = nullptr, *lsi = nullptr, *lbr = nullptr, *lfp = nullptr, *lbp = nullptr;
  if constexpr (STAGE) {
    ltg = reinterpret_cast<int4*>(smem + direct_stage_offset(NBP, NW, d));
    lct = ltg + d.n_tg;
    lje = lct + d.n_ct;
    lso = reinterpret_cast<int*>(lje + d.n_je);
    lsi = lso + m + 1;
    lbr = lsi + ns;
    lfp = lbr + m;
    lbp = lfp + d.n_fph + 1;
    for (int q = tid; q < d.n_tg; q += BLOCK) ltg[q] = cld(d.ftg, (unsigned)q);
    for (int q = tid; q < d.n_ct; q += BLOCK) lct[q] = cld(d.fct, (unsigned)q);
    for (int q = tid; q < d.n_je; q += BLOCK) lje[q] = cld(d.je, (unsigned)q);
    for (int q = tid; q <= m; q += BLOCK) lso[q] = cld(d.soff, (unsigned)q);
    for (int q = tid; q < ns; q += BLOCK) lsi[q] = cld(d.sidx, (unsigned)q);
    for (int q = tid; q < m; q += BLOCK) lbr[q] = cld(d.brow, (unsigned)q);
    for (int q = tid; q <= d.n_fph; q += BLOCK) lfp[q] = cld(d.fph, (unsigned)q);
    for (int q = tid; q <= d.n_bph; q += BLOCK) lbp[q] = cld(d.bph, (unsigned)q);
    // (made visible by the barriers of the first mismatch)
  }
  auto TG = [&](int q) { if constexpr (STAGE) return ltg[q]; else return cld(d.ftg, (unsigned)q); };
  auto CT = [&](int q) { if constexpr (STAGE) return lct[q]; else return cld(d.fct, (unsigned)q); };
  auto JE = [&](int q) { if constexpr (STAGE) return lje[q]; else return cld(d.je, (unsigned)q); };
  auto SO = [&](int q) { if constexpr (STAGE) return lso[q]; else return cld(d.soff, (unsigned)q); };
  auto SI = [&](int q) { if constexpr (STAGE) return lsi[q]; else return cld(d.sidx, (unsigned)q); };
  auto BR = [&](int q) { if constexpr (STAGE) return lbr[q]; else return cld(d.brow, (unsigned)q); };
  auto FPH = [&](int q) { if constexpr (STAGE) return lfp[q]; else return cld(d.fph, (unsigned)q); };
  auto BPH = [&](int q) { if constexpr (STAGE) return lbp[q]; else return cld(d.bph, (unsigned)q); };

  const Ws<BLOCK, KB> ws{make_buf(a.ws_d + (int64_t)b * a.ws_d_stride)};
  const Buf P = make_buf(a.p_inj + (int64_t)b * a.ld);
  const Buf Q = make_buf(a.q_inj + (int64_t)b * a.ld);
  const Buf VS = make_buf(a.vm_set + (int64_t)b * a.ld);
  {
    const TxDev<double> net = load_desc(netp);
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const unsigned i = row<BLOCK>(k);
      double p = 0.0, q = 0.0, vsp = 1.0;
      if ((int)i < n) {
        const unsigned e = (unsigned)cld(net.int2ext, i) * 8u;
        p = bld<double>(P, e, 0);
        q = bld<double>(Q, e, 0);
        if ((int)i >= npq) vsp = bld<double>(VS, e, 0);
      }
      ws.st(TH, k, 0.0);
      ws.st(VM, k, vsp);
      ws.st(PIN, k, p);
      ws.st(QIN, k, q);
    }
  }
  const double2* yv = a.yv64 ? a.yv64 + (int64_t)b * a.yv_stride : nullptr;

  int newton = 0;
  bool conv = false;
  double fnorm = 0.0, work = 0.0;
  int par = 0;
  for (;;) {
    fnorm = mismatch<double, BLOCK, KB>(netp, ws, vs, red + par * NW, yv);
    work += 32.0 * n + 16.0 * m + 16.0 * a.yv_nnz;
    par ^= 1;
    if (!(fnorm <= a.diverge)) break;
    if (fnorm <= a.tol) {
      conv = true;
      break;
    }
    if (newton >= a.max_newton) break;
    // own buses' I and -F into LDS (F in factor order); factor values cleared
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const unsigned i = row<BLOCK>(k);
      is[i] = make_double2(ws.ld(IRE, k), ws.ld(IIM, k));
      if ((int)i < nth) rhs[cld(d.fpos, i)] = -ws.ld(FP, k);
      if ((int)i < npq) rhs[cld(d.fpos, (unsigned)NBP + i)] = -ws.ld(FP, KB + k);
    }
    for (int q = tid; q < d.n_val; q += BLOCK) val[q] = 0.0;
    __syncthreads();
    {
      const TxDev<double> net = load_desc(netp);
      const double2* yvals = yv ? yv : net.y64.val;
      for (int e = tid; e < d.n_je; e += BLOCK) {
        const int4 E = JE(e);
        const int pos = E.x & 0x0fffffff, kind = (int)((unsigned)E.x >> 28);
        const double2 vi = vs[E.y], vk = vs[E.z], y = cld(yvals, (unsigned)E.w);
        const double tr = y.x * vk.x - y.y * vk.y, ti = y.x * vk.y + y.y * vk.x;  // Y_ik V_k
        double ar = vi.x * tr + vi.y * ti, ai = vi.y * tr - vi.x * ti;            // V_i conj(Y_ik V_k)
        double dtr, dti, dvr, dvi;
        if (E.y != E.z) {
          const double ivk = 1.0 / sqrt(vk.x * vk.x + vk.y * vk.y);
          dtr = ai;
          dti = -ar;
          dvr = ar * ivk;
          dvi = ai * ivk;
        } else {
          const double2 ii = is[E.y];
          const double cr = vi.x * ii.x + vi.y * ii.y, ci = vi.y * ii.x - vi.x * ii.y;
          const double ivi = 1.0 / sqrt(vi.x * vi.x + vi.y * vi.y);
          dtr = -(ci - ai);
          dti = cr - ar;
          dvr = (ar + cr) * ivi;
          dvi = (ai + ci) * ivi;
        }
        val[pos] = kind == 0 ? dtr : kind == 1 ? dvr : kind == 2 ? dti : dvi;
      }
    }
    __syncthreads();
    // LU with the forward solve L y = -F fused in, by levels of the
    // elimination tree: one phase per level, one thread per target, which
    // subtracts L[i][k] x / U[k][k] for each of its contributions (pivots of
    // the level, in pivot order; x the U entry or rhs[k]).  Pivots of a level
    // read only their own row, column and rhs entry, which no pivot of the
    // level changes, and L stays unscaled (its entries hold L U[k][k]).
    for (int ph = 0; ph < d.n_fph; ++ph) {
      const int q1 = FPH(ph + 1);
      for (int q = FPH(ph) + tid; q < q1; q += BLOCK) {
        const int4 T = TG(q);
        double acc = 0.0;
        for (int c = T.y; c < T.z; ++c) {
          const int4 C = CT(c);
          acc += val[C.x] * (T.w ? rhs[C.y] : val[C.y]) / val[C.z];
        }
        if (T.w) rhs[T.x] -= acc;
        else val[T.x] -= acc;
      }
      __syncthreads();
    }
    // backward: U x = y by levels, one thread per row: x_k = (y_k - U[k][S(k)]
    // x[S(k)]) / U[k][k], the x it reads solved in earlier levels
    for (int ph = 0; ph < d.n_bph; ++ph) {
      const int q1 = BPH(ph + 1);
      for (int q = BPH(ph) + tid; q < q1; q += BLOCK) {
        const int k = BR(q);
        const int s1 = SO(k + 1);
        double acc = rhs[k];
        for (int t = SO(k); t < s1; ++t) acc -= val[m + ns + t] * xs[SI(t)];
        xs[k] = acc / val[k];
      }
      __syncthreads();
    }
    // Newton update (eq. (3)), own buses
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const unsigned i = row<BLOCK>(k);
      if ((int)i < nth) ws.st(TH, k, ws.ld(TH, k) + xs[cld(d.fpos, i)]);
      if ((int)i < npq) ws.st(VM, k, ws.ld(VM, k) + xs[cld(d.fpos, (unsigned)NBP + i)]);
    }
    work += 8.0 * m + 32.0 * m;
    ++newton;
  }

  const Buf vout = make_buf(a.v_out + 2 * (int64_t)b * a.ld);
  {
    const TxDev<double> net = load_desc(netp);
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const unsigned i = row<BLOCK>(k);
      if ((int)i < n) {
        const unsigned e = (unsigned)cld(net.int2ext, i) * 16u;
        double sn, cs;
        sincos(ws.ld(TH, k), &sn, &cs);
        const double vm = ws.ld(VM, k);
        bst(vout, vm * cs, e, 0);
        bst(vout, vm * sn, e, 8);
      }
    }
  }
  if (tid == 0) {
    a.newton_iters[b] = newton;
    if (a.gmres_iters) a.gmres_iters[b] = 0;
    a.converged[b] = conv ? 1 : 0;
    if (a.final_mismatch) a.final_mismatch[b] = fnorm;
    if (a.work_bytes) a.work_bytes[b] = work;
  }
}

// ---------------------------------------------------------------------------
// Adjoint.  For w = [w_P on Theta ; w_Q on Q] and c = w_P + j w_Q (zero where
// undefined), w^T dF = Re sum_k g_k dV_k with g = conj(c I) + Ybus^T (c conj V),
// so (J^T w) = [-Im(g V) on Theta ; Re(g V) / |V| on Q].  Ends with a barrier.
template <int BLOCK, int KB>
__device__ void vjp(const TxDev<double>* netp, const Ws<BLOCK, KB>& ws, double (&w)[2 * KB], double* lds) {
  constexpr int NW = BLOCK / WAVE;
  const TxDev<double> net = load_desc(netp);
  const unsigned nth = net.nth, npq = net.npq;
  double2* u = reinterpret_cast<double2*>(lds);
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    const unsigned i = row<BLOCK>(k);
    const double cr = w[k], ci = w[KB + k];
    const double vr = ws.ld(VRE, k), vi = ws.ld(VIM, k);
    double2 t;  // c conj(V)
    t.x = cr * vr + ci * vi;
    t.y = ci * vr - cr * vi;
    u[i] = t;
  }
  __syncthreads();
  const int wv = wave_id();
  double nIr = ws.ld(IRE, 0), nIi = ws.ld(IIM, 0), nvr = ws.ld(VRE, 0), nvi = ws.ld(VIM, 0), niv = ws.ld(IVM, 0);
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    const double Ir = nIr, Ii = nIi, vr = nvr, vi = nvi, iv = niv;
    if (k + 1 < KB) {
      nIr = ws.ld(IRE, k + 1);
      nIi = ws.ld(IIM, k + 1);
      nvr = ws.ld(VRE, k + 1);
      nvi = ws.ld(VIM, k + 1);
      niv = ws.ld(IVM, k + 1);
    }
    double gr = 0.0, gi = 0.0;  // (Y^T (c conj V))_i
    psell_row(net.yt, k * NW + wv, [&](double2 y, int c) {
      const double2 t = u[c];
      gr += y.x * t.x - y.y * t.y;
      gi += y.x * t.y + y.y * t.x;
    });
    const unsigned i = row<BLOCK>(k);
    const double cr = w[k], ci = w[KB + k];
    const double hr = gr + cr * Ir - ci * Ii;  // + conj(c I)
    const double hi = gi - (cr * Ii + ci * Ir);
    const double pr = hr * vr - hi * vi, pi = hr * vi + hi * vr;  // g V
    w[k] = i < nth ? -pi : 0.0;
    w[KB + k] = i < npq ? pr * iv : 0.0;
    settle(w[k]);
    settle(w[KB + k]);
  }
  __syncthreads();
}

// z = M^-T w: z_Q = diag(|V_Q|)^-1 (B'' + eps I)^-1 w_Q,
//             z_Theta = diag(|V_Theta|)^-1 (B' + eps I)^-1 (w_Theta - G^T z_Q).
// LDS use as in precond, with the roles of the two solves swapped.
template <int BLOCK, int KB>
__device__ void precond_t(const TxDev<double>* netp, const Ws<BLOCK, KB>& ws, double (&w)[2 * KB],
                          const Smem<double>& s) {
  constexpr int NW = BLOCK / WAVE;
  const TxDev<double> net = load_desc(netp);
  const unsigned nth = net.nth, npq = net.npq;
  double* X = s.xs;
  double* Y = s.xs + nth;
  if (npq > 0) {
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const unsigned i = row<BLOCK>(k);
      if (i < npq) Y[i] = w[KB + k];
    }
    __syncthreads();
    efac_apply<double, BLOCK, KB, KB>(net.bpp, Y, X, s.tmp, w);
#pragma unroll
    for (int k = 0; k < KB; ++k) w[KB + k] *= ws.ld(IVM, k);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const unsigned i = row<BLOCK>(k);
      if (i < npq) Y[i] = w[KB + k];
    }
    __syncthreads();
    const TxDev<double> nt = load_desc(netp);
    double gz[KB];
    psell_slots_dot<KB, NW>(nt.gt, Y, gz);
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const unsigned i = row<BLOCK>(k);
      if (i < nth) X[i] = w[k] - gz[k];
    }
  } else {
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const unsigned i = row<BLOCK>(k);
      if (i < nth) X[i] = w[k];
    }
  }
  __syncthreads();
  const TxDev<double> nb = load_desc(netp);
  efac_apply<double, BLOCK, KB, 0>(nb.bp, X, Y, s.tmp, w);
#pragma unroll
  for (int k = 0; k < KB; ++k) w[k] *= ws.ld(IVM, k);
}

template <int BLOCK, int KB>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void adjoint_kernel(
    const TxDev<double>* __restrict__ netp, AdjLaunch a) {
  constexpr int NW = BLOCK / WAVE;
  constexpr int K = 2 * KB;
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = blockIdx.x;
  int n, nth, npq, kmax;
  {
    const TxDev<double> net = load_desc(netp);
    n = net.n;
    nth = net.nth;
    npq = net.npq;
    kmax = net.bp.k > net.bpp.k ? net.bp.k : net.bpp.k;
  }
  const int R = a.restart;
  const NrLayout L = nr_layout(KB * BLOCK, nth, npq, kmax, R, NW, 8);
  const Smem<double> s = carve<double>(smem, L);
  const Ws<BLOCK, KB> ws{make_buf(a.ws_d + (int64_t)b * a.ws_d_stride)};
  const Basis<double, BLOCK, KB> basis{make_buf(a.ws_basis + (int64_t)b * a.ws_b_stride)};
  const Buf V = make_buf(a.v + 2 * (int64_t)b * a.ld);
  const Buf tg = make_buf(a.dl_dv + 2 * (int64_t)b * a.ld);

  // V, |V|, 1/|V| at the given voltages (padding buses: V = 1)
  {
    const TxDev<double> net = load_desc(netp);
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const unsigned i = row<BLOCK>(k);
      double2 v;
      v.x = 1.0;
      v.y = 0.0;
      if ((int)i < n) {
        const unsigned e = (unsigned)cld(net.int2ext, i) * 16u;
        v.x = bld<double>(V, e, 0);
        v.y = bld<double>(V, e, 8);
      }
      const double vm = sqrt(v.x * v.x + v.y * v.y);
      ws.st(VRE, k, v.x);
      ws.st(VIM, k, v.y);
      ws.st(VM, k, vm);
      ws.st(IVM, k, 1.0 / vm);
      s.vs[i] = v;
    }
  }
  __syncthreads();
  // I = Ybus V, and dL/dx from the torch-convention gradient t = dL/dRe V + j dL/dIm V:
  // dL/dtheta = Im(t) Re(V) - Re(t) Im(V), dL/d|V| = (Re(t) Re(V) + Im(t) Im(V)) / |V|
  {
    const TxDev<double> net = load_desc(netp);
    double Ir[KB], Ii[KB];
#pragma unroll
    for (int k = 0; k < KB; ++k) Ir[k] = Ii[k] = 0.0;
    psell_slots<KB, NW>(
        net.y64,
        [&](int k, double2 y, int c) {
          const double2 v = s.vs[c];
          Ir[k] += y.x * v.x - y.y * v.y;
          Ii[k] += y.x * v.y + y.y * v.x;
        },
        [&](int) {});
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const unsigned i = row<BLOCK>(k);
      ws.st(IRE, k, Ir[k]);
      ws.st(IIM, k, Ii[k]);
      double ft = 0.0, fv = 0.0;
      if ((int)i < n) {
        const unsigned e = (unsigned)cld(net.int2ext, i) * 16u;
        const double tr = bld<double>(tg, e, 0), ti = bld<double>(tg, e, 8);
        const double2 v = s.vs[i];
        if ((int)i < nth) ft = ti * v.x - tr * v.y;
        if ((int)i < npq) fv = (tr * v.x + ti * v.y) * ws.ld(IVM, k);
      }
      ws.st(FP, k, ft);
      ws.st(FP, KB + k, fv);
    }
  }
  __syncthreads();

  auto apply_jt = [&](double (&w)[K]) { vjp<BLOCK, KB>(netp, ws, w, s.xs); };
  auto apply_mt = [&](double (&w)[K]) { precond_t<BLOCK, KB>(netp, ws, w, s); };
  double work = 0.0;
  bool ok;
  int its;
  {
    const TxDev<double> net = load_desc(netp);
    const ByteModel bm{8.0 * net.m, 8.0 * net.m, 8.0 * n, 32.0 * n};
    its = gmres_solve<double, BLOCK, KB>(apply_jt, apply_mt, ws, FP, DXP, basis, R, a.max_restarts, a.rtol, s,
                                         &ok, bm, &work);
  }
  const Buf gp = make_buf(a.grad_p + (int64_t)b * a.ld);
  const Buf gq = make_buf(a.grad_q + (int64_t)b * a.ld);
  // rows that carry no state (the slack's P, the Q of PV buses and the slack) are zero
  {
    const TxDev<double> net = load_desc(netp);
#pragma unroll
    for (int k = 0; k < KB; ++k) {
      const unsigned i = row<BLOCK>(k);
      if ((int)i < n) {
        const unsigned e = (unsigned)cld(net.int2ext, i) * 8u;
        bst(gp, (int)i < nth ? ws.ld(DXP, k) : 0.0, e, 0);
        bst(gq, (int)i < npq ? ws.ld(DXP, KB + k) : 0.0, e, 0);
      }
    }
  }
  if (threadIdx.x == 0) {
    if (a.gmres_iters) a.gmres_iters[b] = its;
    if (a.converged) a.converged[b] = ok ? 1 : 0;
  }
}

// Shapes: BLOCK threads, KB bus slots per thread, n <= BLOCK * KB.
template <typename Launch>
void dispatch_shape(int n, Launch&& go) {
  if (n <= 64) go.template operator()<64, 1>();
  else if (n <= 256) go.template operator()<64, 4>();
  else if (n <= 1024) go.template operator()<256, 4>();
  else if (n <= 2048) go.template operator()<256, 8>();
  else if (n <= 4096) go.template operator()<512, 8>();
  else if (n <= 8192) go.template operator()<1024, 8>();
  else fail(PF_INVALID_ARG, "networks above 8192 buses are not supported");
}

struct ShapeOf {
  int* block;
  int* kb;
  template <int BLOCK, int KB>
  void operator()() const {
    *block = BLOCK;
    *kb = KB;
  }
};

size_t lds_bytes(const TxNetwork& net, int R, int ts) {
  const int kmax = std::max(net.bp.host.k, net.bpp.host.k);
  const NrLayout L = nr_layout(net.nbp, net.nth, net.npq, kmax, R, net.block / WAVE, ts);
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
  template <int BLOCK, int KB>
  void operator()() const {
    const size_t lds = lds_bytes(net, a.restart, (int)sizeof(T));
    auto kernel = nr_kernel<T, BLOCK, KB>;
    if (lds > 64 * 1024)
      PFX_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(kernel, dim3(a.batch), dim3(BLOCK), lds, s, net.desc<T>(), a);
    PFX_HIP(hipGetLastError());
  }
};

struct NrDirectGo {
  const TxNetwork& net;
  const NRLaunch& a;
  hipStream_t s;
  template <int BLOCK, int KB>
  void operator()() const {
    const DirectDev& d = net.direct;
    const size_t lds0 = (size_t)2 * KB * BLOCK * 16 + 2 * (BLOCK / WAVE) * 8 + ((size_t)d.n_val + 2 * d.m) * 8;
    if (lds0 > 160 * 1024) {
      // factor values in device memory; V, I, the right-hand side and x stay in LDS
      const size_t ldsg = (size_t)2 * KB * BLOCK * 16 + 2 * (BLOCK / WAVE) * 8 + (size_t)2 * d.m * 8;
      if (ldsg > 160 * 1024)
        fail(PF_INVALID_ARG, "network too large for the direct Newton step (" + std::to_string(ldsg) +
                                 " bytes of LDS)");
      if (!a.ws_dval) fail(PF_INVALID_ARG, "direct Newton step without its factor workspace");
      auto kernel = nr_direct_kernel<BLOCK, KB, false, true>;
      if (ldsg > 64 * 1024)
        PFX_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)ldsg));
      hipLaunchKernelGGL(kernel, dim3(a.batch), dim3(BLOCK), ldsg, s, net.desc<double>(), d, a);
      PFX_HIP(hipGetLastError());
      return;
    }
    // stage the schedule tables when the total stays within 64 KB, or, when
    // the batch has no more scenarios than the chip has CUs (one workgroup
    // per CU, occupancy moot), within the CU's 160 KB
    const size_t lds1 = direct_stage_offset(KB * BLOCK, BLOCK / WAVE, d) + direct_stage_bytes(d);
    const bool stage = lds1 <= (a.batch <= net.ctx->cu_count ? 160 : 64) * 1024;
    const size_t lds = stage ? lds1 : lds0;
    auto kernel = stage ? nr_direct_kernel<BLOCK, KB, true, false> : nr_direct_kernel<BLOCK, KB, false, false>;
    if (lds > 64 * 1024)
      PFX_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(kernel, dim3(a.batch), dim3(BLOCK), lds, s, net.desc<double>(), d, a);
    PFX_HIP(hipGetLastError());
  }
};

struct AdjGo {
  const TxNetwork& net;
  const AdjLaunch& a;
  hipStream_t s;
  template <int BLOCK, int KB>
  void operator()() const {
    const size_t lds = lds_bytes(net, a.restart, 8);
    auto kernel = adjoint_kernel<BLOCK, KB>;
    if (lds > 64 * 1024)
      PFX_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(kernel, dim3(a.batch), dim3(BLOCK), lds, s, net.desc<double>(), a);
    PFX_HIP(hipGetLastError());
  }
};

}  // namespace

void nr_shape(int n, int* block, int* kb) { dispatch_shape(n, ShapeOf{block, kb}); }

int64_t nr_padded_rows(const TxNetwork& net) { return 2 * (int64_t)net.nbp; }
int64_t nr_ws_doubles(const TxNetwork& net) { return 13 * (int64_t)net.nbp; }
int64_t adj_ws_doubles(const TxNetwork& net) { return nr_ws_doubles(net); }

// One thread per (scenario, layout entry), grid-stride over the batch.
__global__ __launch_bounds__(256) void y_gather_kernel(const int* sptr, const int* sidx, int64_t E, int batch,
                                                       const double* yv, int64_t ldy, double2* out64,
                                                       float2* out32) {
  const int64_t total = E * batch;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < total; t += (int64_t)gridDim.x * 256) {
    const int64_t b = t / E, q = t - b * E;
    const double* src = yv + 2 * ldy * b;
    double re = 0.0, im = 0.0;
    for (int k = sptr[q]; k < sptr[q + 1]; ++k) {
      const int e = sidx[k];
      re += src[2 * e];
      im += src[2 * e + 1];
    }
    out64[t] = make_double2(re, im);
    if (out32) out32[t] = make_float2((float)re, (float)im);
  }
}

void launch_y_gather(const TxNetwork& net, int batch, int64_t ldy, const double* y_vals, double2* yv64,
                     float2* yv32, hipStream_t s) {
  if (batch == 0 || net.y_entries == 0) return;
  const int64_t total = net.y_entries * batch;
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(y_gather_kernel, dim3((unsigned)blocks), dim3(256), 0, s, net.ysrc_ptr.as<int>(),
                     net.ysrc_idx.as<int>(), net.y_entries, batch, y_vals, ldy, yv64, yv32);
  PFX_HIP(hipGetLastError());
}

void launch_nr(const TxNetwork& net, bool mixed, const NRLaunch& a, hipStream_t s) {
  if (a.batch == 0) return;
  if (mixed) dispatch_shape(net.n, NrGo<float>{net, a, s});
  else dispatch_shape(net.n, NrGo<double>{net, a, s});
}

bool direct_lds_fits(const TxNetwork& net) {
  const DirectDev& d = net.direct;
  const size_t lds0 = (size_t)2 * net.nbp * 16 + 2 * (net.block / WAVE) * 8 + ((size_t)d.n_val + 2 * d.m) * 8;
  return lds0 <= 160 * 1024;
}

void launch_nr_direct(const TxNetwork& net, const NRLaunch& a, hipStream_t s) {
  if (a.batch == 0) return;
  if (!net.direct_ready) fail(PF_INVALID_ARG, "direct Newton step used before its analysis was built");
  dispatch_shape(net.n, NrDirectGo{net, a, s});
}

void launch_adjoint(const TxNetwork& net, const AdjLaunch& a, hipStream_t s) {
  if (a.batch == 0) return;
  dispatch_shape(net.n, AdjGo{net, a, s});
}

// ---------------------------------------------------------------------------
// Branch-current loss L = sum_f |I_f|^2, I_f = (y_s + j b/2) V_f - y_s V_t,
// and dL/dV in torch's convention conj(g), g_k = dL/dV_k (complex derivative).
// One workgroup per scenario; the gradient is accumulated per bus by walking
// each bus's incident branches (no atomics, fixed order).
__global__ __launch_bounds__(256) void branch_loss_kernel(const TxDev<double>* __restrict__ netp,
                                                          const int* inc_ptr, const int* inc_br, LossLaunch a) {
  __shared__ double red[4];
  const TxDev<double> net = load_desc(netp);
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
