// Batched three-phase Z-bus fixed point (Sec. II-B, eq. (10)).
//
// The iteration is run in residual form: with r = i(v) - (Y_NN v + Y_NS v_S),
//   v <- v + Z r,
// which equals Z i(v) + v0 exactly because Z (Y_NN v + Y_NS v_S) = v - v0.  The
// residual, the power mismatch v * conj(r), the convergence test and the
// update are FP64; the product Z r runs on the matrix cores in FP64, or in
// FP32 with FP32 accumulation in mixed mode (the FP64 residual then drives the
// FP32 error to zero as r -> 0).
//
// Kernels per iteration:
//   zb_residual   one workgroup per scenario: wye and delta load currents,
//                 sparse Y_NN v (sliced ELLPACK, v staged in LDS), r,
//                 max |v * conj(r)|, flags, sum |v|
//   zb_gemm_*     D = R W (real-block form of Z r) on MFMA 16x16x4 tiles, with
//                 the FP64 update v += D fused into the epilogue (FP64:
//                 operands straight from memory; FP32: staged through LDS)
//   zb_sparse     (sparse variant, instead of the GEMM) v += Y_NN^-1 r by
//                 level-scheduled solves with the sparse L D L^T of Y_NN
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <type_traits>

#include "device_ops.hpp"
#include "dist.hpp"

namespace pfx {

namespace {

// Complex values of per-scenario rows: one 16-byte load or an 8/16-byte store.
typedef double D2 __attribute__((ext_vector_type(2)));
typedef float F2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ D2 ld2(const double* base, unsigned i) {
  typedef __attribute__((address_space(1))) const D2 GD2;
  return ((GD2*)base)[i];
}

__device__ __forceinline__ void st2(double* base, unsigned i, double x, double y) {
  typedef __attribute__((address_space(1))) D2 GD2;
  ((GD2*)base)[i] = D2{x, y};
}

__device__ __forceinline__ void st2(float* base, unsigned i, double x, double y) {
  typedef __attribute__((address_space(1))) F2 GF2;
  ((GF2*)base)[i] = F2{(float)x, (float)y};
}

// conj(s / v) for complex s, v
__device__ __forceinline__ D2 conj_div(D2 s, double vr, double vi) {
  const double d = vr * vr + vi * vi;
  return D2{(s.x * vr + s.y * vi) / d, -(s.y * vr - s.x * vi) / d};
}

constexpr int WYE_BIT = 1 << 30;

__device__ __forceinline__ int zb_slot(const ZbusLaunch& a, int g) { return a.slots ? a.slots[g] : g; }

__global__ __launch_bounds__(ZB_THREADS) void zb_init(DistDev net, ZbusLaunch a) {
  const int b = zb_slot(a, blockIdx.x);
  double* v = a.v + (int64_t)b * net.Kp;
  for (int i = threadIdx.x; i < 2 * net.nN; i += ZB_THREADS) v[i] = net.v0[i];
  // the per-iteration active counts start at zero (a fill here rather than a
  // memset node, so the solve can be captured into a graph)
  if (blockIdx.x == 0 && a.count)
    for (int i = threadIdx.x; i <= a.max_iter; i += ZB_THREADS) a.count[i] = 0;
  if (threadIdx.x == 0) {
    a.active[b] = 1;
    a.iters[b] = 0;
    a.converged[b] = 0;
    a.st[3 * b + 0] = 0.0;
    a.st[3 * b + 1] = 0.0;
    a.st[3 * b + 2] = 0.0;
  }
}

// One workgroup per scenario; wave w owns node slices k * 4 + w (k < KB).
// Per node: the load current i(v) (wye: -conj(S / v); delta: the two branch
// currents of the node's delta), the row of Y_NN v + c from the sliced
// ELLPACK copy of Y_NN (entries read in rounds of 4), the residual r (stored
// in the GEMM's type), |v conj(r)| and |v|.  The workgroup's max and sum are
// finished by thread 0, which also sets the scenario's flags.
template <typename T, int KB>
__global__ __launch_bounds__(ZB_THREADS) __attribute__((amdgpu_waves_per_eu(8))) void zb_residual(
    DistDev net, ZbusLaunch a, int it) {
  constexpr int NW = ZB_THREADS / WAVE;
  extern __shared__ D2 vs[];  // [nNs]
  __shared__ double red[2][NW];
  const int g = blockIdx.x;
  // whole-batch solves: nothing to do once the previous iteration left no
  // scenario active (all iterations may be enqueued at once)
  if (a.count && it > 0 && a.count[it - 1] == 0) return;
  const int b = zb_slot(a, g);
  if (a.active[b] == 0) {
    if (a.step_done && threadIdx.x == 0) a.step_done[g] = 1;
    return;
  }
  const int nN = net.nN, nNs = net.nNs;
  const double* vrow = a.v + (int64_t)b * net.Kp;
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    const unsigned i = threadIdx.x + k * ZB_THREADS;
    if (i < (unsigned)nNs) vs[i] = i < (unsigned)nN ? ld2(vrow, i) : D2{0.0, 0.0};
  }
  __syncthreads();
  const double* SW = a.s_wye + 2 * (int64_t)b * a.ld;
  const double* SD = a.s_delta + 2 * (int64_t)b * a.ld;
  T* r = reinterpret_cast<T*>(a.r) + (int64_t)g * net.Kp;
  const int wv = wave_id(), lane = lane_id();
  double mm = 0.0, sabs = 0.0;
#pragma unroll
  for (int k = 0; k < KB; ++k) {
    const int sl = k * NW + wv;
    if (sl * WAVE >= nNs) break;
    const unsigned i = (unsigned)(sl * WAVE + lane);
    const int4 nd = cld(net.node, i);
    const double2 c = cld(net.c, i);
    double yr = c.x, yi = c.y;
    const int o = cld(net.y.off, (unsigned)sl);
    const int wd = cld(net.y.width, (unsigned)sl);
    int p = 0;
    for (; p + 8 <= wd; p += 8) {  // eight entries in flight per round while they last
      double2 g[8];
      int cj[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const unsigned q = (unsigned)(o + (p + u) * WAVE + lane);
        g[u] = cld(net.y.val, q);
        cj[u] = cld(net.y.col, q);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const D2 x = vs[cj[u]];
        yr += g[u].x * x.x - g[u].y * x.y;
        yi += g[u].x * x.y + g[u].y * x.x;
      }
    }
    if (p < wd) {  // widths are multiples of 4: at most one round of four remains
      double2 g[4];
      int cj[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const unsigned q = (unsigned)(o + (p + u) * WAVE + lane);
        g[u] = cld(net.y.val, q);
        cj[u] = cld(net.y.col, q);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const D2 x = vs[cj[u]];
        yr += g[u].x * x.x - g[u].y * x.y;
        yi += g[u].x * x.y + g[u].y * x.x;
      }
    }
    const int e = nd.x & (WYE_BIT - 1);
    D2 sw = {0.0, 0.0}, sx = {0.0, 0.0}, sp = {0.0, 0.0};
    if (nd.x & WYE_BIT) sw = ld2(SW, (unsigned)e);
    if (nd.y >= 0) {
      sx = ld2(SD, (unsigned)e);
      sp = ld2(SD, (unsigned)nd.w);
    }
    if (i < (unsigned)nN) {
      const D2 v = vs[i];
      double ir = 0.0, ii = 0.0;
      if (nd.x & WYE_BIT) {
        const D2 q = conj_div(sw, v.x, v.y);
        ir -= q.x;
        ii -= q.y;
      }
      if (nd.y >= 0) {  // branch x->next carries S_x, branch prev->x carries S_prev
        const D2 vn = vs[nd.y], vp = vs[nd.z];
        const D2 ax = conj_div(sx, v.x - vn.x, v.y - vn.y);
        const D2 ap = conj_div(sp, vp.x - v.x, vp.y - v.y);
        ir -= ax.x - ap.x;
        ii -= ax.y - ap.y;
      }
      const double rr = ir - yr, ri = ii - yi;
      const double dr = v.x * rr + v.y * ri, di = v.y * rr - v.x * ri;  // v conj(r)
      mm = nanmax(mm, sqrt(dr * dr + di * di));
      sabs += sqrt(v.x * v.x + v.y * v.y);
      st2(r, i, rr, ri);
    }
  }
  mm = wave_nanmax(mm);
  sabs = wave_total(sabs);
  if (lane == 0) {
    red[0][wv] = mm;
    red[1][wv] = sabs;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    mm = red[0][0];
    sabs = red[1][0];
#pragma unroll
    for (int w = 1; w < NW; ++w) {
      mm = nanmax(mm, red[0][w]);
      sabs += red[1][w];
    }
    if (a.slots) it = a.iters[b];
    double* st = a.st + 3 * (int64_t)b;
    st[0] = mm;
    if (it > 0) st[2] = fabs(sabs - st[1]);
    st[1] = sabs;
    int more = 0;
    if (mm <= a.tol) {
      a.converged[b] = 1;
      a.active[b] = 0;
    } else if (!(mm == mm) || it >= a.max_iter) {
      a.active[b] = 0;
    } else {
      a.iters[b] = it + 1;
      more = 1;
      if (a.count) atomicAdd(&a.count[it], 1);
    }
    if (a.step_done) a.step_done[g] = more ? 0 : 1;
  }
}

template <typename T>
struct Mfma;

// Lane layouts of the 16x16x4 MFMA tiles (measured on gfx950): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; the four accumulator values of lane l
// hold column l % 16 of rows out_row(l, v).  The FP64 form interleaves rows
// (v picks the row group), the FP32 form keeps four consecutive rows.
template <>
struct Mfma<double> {
  typedef double V4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ V4 op(double x, double y, V4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int lane, int v) { return 4 * v + lane / 16; }
};

template <>
struct Mfma<float> {
  typedef float V4 __attribute__((ext_vector_type(4)));
  static __device__ __forceinline__ V4 op(float x, float y, V4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int out_row(int lane, int v) { return 4 * (lane / 16) + v; }
};

// FP32 form (mixed precision): D = R W on a ZB_BM x ZB_BN tile per
// workgroup (4 waves, 2 x 2, 64 x 64 each, 4 x 4 MFMA 16x16x4 tiles per
// wave), K in steps of ZB_BK staged through LDS, double buffered; W row-major
// (Kp x Np).  Epilogue: v += D for active scenarios (FP64).
//
// LDS rows are padded by 16 elements so that the four row groups a fragment
// read touches (one per 16 lanes) start in different banks.  Two workgroups
// per CU (two waves per SIMD) keep the matrix pipe busy while the other wave
// waits on LDS or memory: the 4 x 4 accumulator tiles (64 values per lane)
// and the two staging register sets must fit in half the register file.
constexpr int ZB_PAD = 16;

template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void zb_gemm_lds(
    DistDev net, const T* __restrict__ W, ZbusLaunch a, int it) {
  using V4 = typename Mfma<T>::V4;
  const int Kp = net.Kp, Np = net.Np;
  __shared__ T As[2][ZB_BK][ZB_BM + ZB_PAD];
  __shared__ T Bs[2][ZB_BK][ZB_BN + ZB_PAD];
  // Workgroups are dealt to the 8 XCDs round robin (workgroup id mod 8).  When
  // the tile count divides by 8, XCD x gets the contiguous tile range
  // [x T/8, (x+1) T/8) in row-major tile order, so the R rows of a tile row
  // are read into one XCD's L2 and W streams through each L2 once.
  const int nt = Np / ZB_BN, ntiles = gridDim.x;
  const int id = blockIdx.x;
  const int lin = (ntiles & 7) == 0 ? (id & 7) * (ntiles >> 3) + (id >> 3) : id;
  const int tile_n = lin % nt, tile_m = lin / nt;
  const int row0 = tile_m * ZB_BM, col0 = tile_n * ZB_BN;
  const int t = threadIdx.x;
  if (a.count && a.count[it] == 0) return;  // no scenario left active (uniform)
  {
    int act = 0;
    if (t < ZB_BM && row0 + t < a.batch) act = a.active[zb_slot(a, row0 + t)];
    if (!__syncthreads_or(act)) return;
  }
  const T* R = reinterpret_cast<const T*>(a.r);
  const int lane = t & (WAVE - 1), wave = t / WAVE;
  const int wm = wave >> 1, wn = wave & 1;
  // global -> LDS assignment: A: row t/2, 8 values from column (t&1)*8; B: row t/16, 8 from (t&15)*8
  const int ar = t >> 1, ac = (t & 1) * 8;
  const int br = t >> 4, bc = (t & 15) * 8;
  const T* Ag = R + (int64_t)(row0 + ar) * Kp + ac;
  const T* Bg = W + (int64_t)br * Np + col0 + bc;

  V4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = V4{0, 0, 0, 0};

  // Global tiles are prefetched two K steps ahead into two register sets
  // (tile j goes through set j & 1), LDS is double buffered (tile j in
  // buffer j & 1): a tile's loads have a whole K step of MFMAs to land.
  T ra[2][8], rb[2][8];
  auto gload = [&](int kt, int set) {
#pragma unroll
    for (int q = 0; q < 8; ++q) ra[set][q] = Ag[kt * ZB_BK + q];
#pragma unroll
    for (int q = 0; q < 8; ++q) rb[set][q] = Bg[(int64_t)kt * ZB_BK * Np + q];
  };
  auto sstore = [&](int buf, int set) {
#pragma unroll
    for (int q = 0; q < 8; ++q) As[buf][ac + q][ar] = ra[set][q];
#pragma unroll
    for (int q = 0; q < 8; ++q) Bs[buf][br][bc + q] = rb[set][q];
  };
  auto compute = [&](int buf) {
#pragma unroll
    for (int kk = 0; kk < ZB_BK / 4; ++kk) {
      const int kr = kk * 4 + lane / 16;
      T af[4], bf[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) af[i] = As[buf][kr][wm * 64 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j) bf[j] = Bs[buf][kr][wn * 64 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = Mfma<T>::op(af[i], bf[j], acc[i][j]);
    }
  };
  const int nk = Kp / ZB_BK;
  // one K step on tile kt (in LDS buffer and register set P = kt & 1)
  auto step = [&](int kt, auto par) {
    constexpr int P = decltype(par)::value;
    if (kt + 2 < nk) gload(kt + 2, P);
    compute(P);
    if (kt + 1 < nk) sstore(P ^ 1, P ^ 1);
    __syncthreads();
  };
  gload(0, 0);
  sstore(0, 0);
  if (nk > 1) gload(1, 1);
  __syncthreads();
  for (int kt = 0; kt < nk; kt += 2) {
    step(kt, std::integral_constant<int, 0>{});
    if (kt + 1 < nk) step(kt + 1, std::integral_constant<int, 1>{});
  }
  const int ncol = 2 * net.nN;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int vv = 0; vv < 4; ++vv) {
      const int row = row0 + wm * 64 + i * 16 + Mfma<T>::out_row(lane, vv);
      if (row >= a.batch) continue;
      const int sc = zb_slot(a, row);
      if (a.active[sc] == 0) continue;
      double* vrow = a.v + (int64_t)sc * Kp;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int col = col0 + wn * 64 + j * 16 + (lane & 15);
        if (col < ncol) vrow[col] += (double)acc[i][j][vv];
      }
    }
  }
}

// FP64 form: D = R W on a ZB_BM x ZB_BN tile per workgroup (4 waves, 2 x 2,
// 64 x 64 each, 4 x 4 MFMA 16x16x4 tiles per wave).  Epilogue: v += D for
// active scenarios.
//
// No LDS and no barrier in the K loop: each wave loads its own operands
// straight into registers in the MFMA's lane layout.  The sum over a K block
// of 16 may visit k in any order as long as A and B agree, so in the block's
// MFMA number c (0..3) lane group g = lane / 16 supplies k = 4 g + c: a
// lane's four k values are contiguous in R's row, and W is stored in K
// blocks of 16 (element (k, n) at ((k / 16) Np + n) 16 + k % 16) so that
// they are contiguous there too.  Operands arrive in 16-byte loads of CH
// values (a substep: CH MFMAs per tile pair), one substep ahead in a second
// register set.  Two workgroups per CU (two waves per SIMD): the 4 x 4
// accumulator tiles and the two operand sets fit in half the register file.
// (In FP32 a lane's four k values take half a 128-byte line, and the eight
// waves of a CU touch more lines than L1 holds before each line's second
// half is read: the FP32 form keeps the LDS kernel above, which measured
// 275 us against about 440 us for this one at batch 4096.)
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void zb_gemm_direct(
    DistDev net, const T* __restrict__ W, ZbusLaunch a, int it) {
  using V4 = typename Mfma<T>::V4;
  constexpr int CH = 16 / sizeof(T);   // values per 16-byte load
  constexpr int NS = ZB_BK / 4 / CH;   // substeps per K block
  typedef T VC __attribute__((ext_vector_type(CH)));
  typedef __attribute__((address_space(1))) const VC GVC;
  const int Kp = net.Kp, Np = net.Np;
  // Workgroups are dealt to the 8 XCDs round robin (workgroup id mod 8).  When
  // the tile count divides by 8, XCD x gets the contiguous tile range
  // [x T/8, (x+1) T/8) in row-major tile order, so the R rows of a tile row
  // are read into one XCD's L2 and W streams through each L2 once.
  const int nt = Np / ZB_BN, ntiles = gridDim.x;
  const int id = blockIdx.x;
  const int lin = (ntiles & 7) == 0 ? (id & 7) * (ntiles >> 3) + (id >> 3) : id;
  const int tile_n = lin % nt, tile_m = lin / nt;
  const int row0 = tile_m * ZB_BM, col0 = tile_n * ZB_BN;
  const int t = threadIdx.x;
  if (a.count && a.count[it] == 0) return;  // no scenario left active (uniform)
  {
    int act = 0;
    if (t < ZB_BM && row0 + t < a.batch) act = a.active[zb_slot(a, row0 + t)];
    if (!__syncthreads_or(act)) return;
  }
  const T* R = reinterpret_cast<const T*>(a.r);
  const int lane = t & (WAVE - 1), wave = t / WAVE;
  const int wm = wave >> 1, wn = wave & 1;
  const int g = lane >> 4, r = lane & 15;
  // this lane's operand rows: R row (tile row i) and W column (tile column j)
  const T* Ab = R + (int64_t)(row0 + wm * 64 + r) * Kp + 4 * g;
  const T* Bb = W + (int64_t)(col0 + wn * 64 + r) * ZB_BK + 4 * g;
  const int64_t a_i = (int64_t)16 * Kp, b_j = 16 * ZB_BK, b_kb = (int64_t)Np * ZB_BK;

  V4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = V4{0, 0, 0, 0};

  VC ao[2][4], bo[2][4];
  auto load = [&](int u, int set) {  // substep u: K block u / NS, part u % NS
    const int kb = u / NS, q = (u % NS) * CH;
#pragma unroll
    for (int i = 0; i < 4; ++i) ao[set][i] = *(GVC*)(Ab + i * a_i + kb * ZB_BK + q);
#pragma unroll
    for (int j = 0; j < 4; ++j) bo[set][j] = *(GVC*)(Bb + j * b_j + kb * b_kb + q);
  };
  auto compute = [&](int set) {
#pragma unroll
    for (int c = 0; c < CH; ++c)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = Mfma<T>::op(ao[set][i][c], bo[set][j][c], acc[i][j]);
  };
  // Straight-line pairs of substeps; past the last substep the loads repeat
  // it (into a set nothing reads again).  The scheduling barriers keep each
  // substep's loads ahead of the previous substep's products (left alone,
  // the compiler gathers a pair's loads at the top of the pair, so each
  // product waits for a load issued just before it).
  const int nu = Kp / ZB_BK * NS;
  load(0, 0);
  int u = 0;
  for (; u + 2 <= nu; u += 2) {
    load(u + 1, 1);
    __builtin_amdgcn_sched_barrier(0);
    compute(0);
    __builtin_amdgcn_sched_barrier(0);
    load(min(u + 2, nu - 1), 0);
    __builtin_amdgcn_sched_barrier(0);
    compute(1);
    __builtin_amdgcn_sched_barrier(0);
  }
  if (u < nu) compute(0);
  const int ncol = 2 * net.nN;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int vv = 0; vv < 4; ++vv) {
      const int row = row0 + wm * 64 + i * 16 + Mfma<T>::out_row(lane, vv);
      if (row >= a.batch) continue;
      const int sc = zb_slot(a, row);
      if (a.active[sc] == 0) continue;
      double* vrow = a.v + (int64_t)sc * Kp;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int col = col0 + wn * 64 + j * 16 + (lane & 15);
        if (col < ncol) vrow[col] += (double)acc[i][j][vv];
      }
    }
  }
}

// One triangular solve of the sparse variant, in place on u (LDS, factor
// order).  Slices run in order with a barrier after each level's last slice:
// a level's rows read only rows of earlier levels, so its slices need no
// barrier between them.  The next slice's descriptor, row ids, first round of
// entries (and 1 / D) are loaded while the current slice computes, so a
// level's cost is its LDS gathers and barrier rather than a chain of
// dependent loads.  BACK: u_i <- u_i / D_i - sum L^T_ij u_j (with the row's
// 1 / D); otherwise u_i <- u_i - sum L_ij u_j.
template <typename T, bool BACK>
__device__ __forceinline__ void zf_solve(typename Vec2<T>::type* u, int nq, const int4* meta, const int* row,
                                         const int* col, const typename Vec2<T>::type* val,
                                         const typename Vec2<T>::type* dinv) {
  using T2 = typename Vec2<T>::type;
  if (nq == 0) return;
  const int lane = threadIdx.x;
  auto round = [&](int at, T2 (&c)[4], int (&j)[4]) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      c[t] = cld(val, (unsigned)(at + t * WAVE + lane));
      j[t] = cld(col, (unsigned)(at + t * WAVE + lane));
    }
  };
  auto apply = [&](const T2 (&c)[4], const int (&j)[4], T2& acc) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const T2 z = u[j[t]];
      acc.x -= c[t].x * z.x - c[t].y * z.y;
      acc.y -= c[t].x * z.y + c[t].y * z.x;
    }
  };
  // One slice's descriptor, row id, first round of entries and 1 / D.  Two
  // of them alternate (the loop is unrolled by two), so a slice's loads stay
  // in flight while the previous slice computes and no register copy at the
  // loop's back edge waits for them.
  struct Slot {
    int4 m;
    int i;
    T2 c[4], d;
    int j[4];
  };
  auto load = [&](int q, Slot& S) {
    S.m = cld(meta, (unsigned)q);
    S.i = cld(row, (unsigned)(q * WAVE + lane));
    round(S.m.x, S.c, S.j);
    if (BACK) S.d = cld(dinv, (unsigned)(q * WAVE + lane));
  };
  auto run = [&](const Slot& S) {
    const T2 z = u[S.i < 0 ? 0 : S.i];
    T2 acc = z;
    if (BACK) {
      acc.x = z.x * S.d.x - z.y * S.d.y;
      acc.y = z.x * S.d.y + z.y * S.d.x;
    }
    apply(S.c, S.j, acc);
    for (int e = 4; e < S.m.y; e += 4) {
      T2 c2[4];
      int j2[4];
      round(S.m.x + e * WAVE, c2, j2);
      apply(c2, j2, acc);
    }
    if (S.i >= 0) u[S.i] = acc;
    if (S.m.z) wave_lds_sync();  // one wavefront per workgroup (see zb_sparse)
  };
  Slot A, B;
  load(0, A);
  int q = 0;
  for (; q + 1 < nq; q += 2) {
    load(q + 1, B);
    run(A);
    load(q + 2 < nq ? q + 2 : q + 1, A);  // the last pair re-reads a slice it holds
    run(B);
  }
  if (q < nq) run(A);
}

// Sparse variant of the update: v += Y_NN^-1 r by the L D L^T factor of
// Y_NN (zfactor.hpp), one wavefront per active scenario: r is placed into
// factor order in LDS, the forward solve L z = r and the backward solve
// L^T x = D^-1 z run in place, and x is added to v in FP64.  Arithmetic in T
// (FP32 in mixed mode, the FP64 residual then refines the result as for the
// dense product).
template <typename T>
__global__ __launch_bounds__(WAVE) void zb_sparse(DistDev net, ZbusLaunch a, int it) {
  using T2 = typename Vec2<T>::type;
  extern __shared__ __align__(16) unsigned char zsm[];
  T2* u = reinterpret_cast<T2*>(zsm);  // [nN]
  if (a.count && a.count[it] == 0) return;  // no scenario left active
  const int g = blockIdx.x;
  const int b = zb_slot(a, g);
  if (a.active[b] == 0) return;
  const int nN = net.nN, lane = threadIdx.x;
  const T2* r = reinterpret_cast<const T2*>(reinterpret_cast<const T*>(a.r) + (int64_t)g * net.Kp);
  constexpr bool f64 = sizeof(T) == 8;
  for (int i = lane; i < nN; i += WAVE) u[cld(net.zf_pinv, (unsigned)i)] = r[i];
  __syncthreads();
  zf_solve<T, false>(u, net.zf_nfq, net.zf_fmeta, net.zf_frow, net.zf_fcol,
                     f64 ? reinterpret_cast<const T2*>(net.zf_fval64) : reinterpret_cast<const T2*>(net.zf_fval32),
                     nullptr);
  zf_solve<T, true>(u, net.zf_nbq, net.zf_bmeta, net.zf_brow, net.zf_bcol,
                    f64 ? reinterpret_cast<const T2*>(net.zf_bval64) : reinterpret_cast<const T2*>(net.zf_bval32),
                    f64 ? reinterpret_cast<const T2*>(net.zf_bd64) : reinterpret_cast<const T2*>(net.zf_bd32));
  double2* v = reinterpret_cast<double2*>(a.v + (int64_t)b * net.Kp);
  for (int i = lane; i < nN; i += WAVE) {
    const T2 x = u[cld(net.zf_pinv, (unsigned)i)];
    double2 y = v[i];
    y.x += (double)x.x;
    y.y += (double)x.y;
    v[i] = y;
  }
}

__global__ __launch_bounds__(ZB_THREADS) void zb_finish(DistDev net, ZbusLaunch a, const int* slack,
                                                       const double* vslack) {
  const int b = zb_slot(a, blockIdx.x);
  const double* v = a.v + (int64_t)b * net.Kp;
  double* out = a.v_out + 2 * (int64_t)b * a.ld;
  for (int i = threadIdx.x; i < net.nN; i += ZB_THREADS) {
    const int e = net.free2ext[i];
    out[2 * e] = v[2 * i];
    out[2 * e + 1] = v[2 * i + 1];
  }
  if (threadIdx.x < 3) {
    const int e = slack[threadIdx.x];
    out[2 * e] = vslack[2 * threadIdx.x];
    out[2 * e + 1] = vslack[2 * threadIdx.x + 1];
  }
  if (threadIdx.x == 0) {
    if (a.final_mismatch) a.final_mismatch[b] = a.st[3 * (int64_t)b];
    if (a.sum_abs_change) a.sum_abs_change[b] = a.st[3 * (int64_t)b + 2];
  }
}

// The update's GEMM: FP64 without LDS (W in K blocks), FP32 through LDS (W row-major).
template <typename T>
void launch_gemm(const DistDev& d, const T* W, const ZbusLaunch& a, int it, int tiles, hipStream_t s) {
  if constexpr (sizeof(T) == 8)
    hipLaunchKernelGGL(zb_gemm_direct<T>, dim3(tiles), dim3(256), 0, s, d, W, a, it);
  else
    hipLaunchKernelGGL(zb_gemm_lds<T>, dim3(tiles), dim3(256), 0, s, d, W, a, it);
}

template <typename T>
void run_zbus_t(DistNetwork& net, const ZbusLaunch& a, hipStream_t s) {
  const DistDev d = net.view();
  const T* W = sizeof(T) == 8 ? net.W64.as<T>() : net.W32.as<T>();
  const int B = a.batch;
  const int mt = (B + ZB_BM - 1) / ZB_BM;
  const int nt = net.Np / ZB_BN;
  const size_t lds = (size_t)d.nNs * 2 * sizeof(double);
  const int kb_need = (d.nNs + ZB_THREADS - 1) / ZB_THREADS;
  auto residual = kb_need <= 1 ? zb_residual<T, 1>
                  : kb_need <= 2 ? zb_residual<T, 2>
                  : kb_need <= 4 ? zb_residual<T, 4>
                  : kb_need <= 8 ? zb_residual<T, 8>
                                 : zb_residual<T, 16>;
  hipLaunchKernelGGL(zb_init, dim3(B), dim3(ZB_THREADS), 0, s, d, a);
  PFX_HIP(hipGetLastError());
  auto update = [&](int it) {
    if (a.sparse) {
      hipLaunchKernelGGL(zb_sparse<T>, dim3(B), dim3(WAVE), (size_t)d.nN * 2 * sizeof(T), s, d, a, it);
    } else {
      launch_gemm<T>(d, W, a, it, nt * mt, s);
    }
    PFX_HIP(hipGetLastError());
  };
  if (a.async && a.max_iter <= ZB_ASYNC_MAX_ITER) {
    // Every iteration enqueued at once: each kernel first reads the active
    // count its predecessor left and exits when it is zero, so the host
    // never waits and the iterations after convergence cost only their
    // launches.
    for (int it = 0; it <= a.max_iter; ++it) {
      hipLaunchKernelGGL(residual, dim3(B), dim3(ZB_THREADS), lds, s, d, a, it);
      PFX_HIP(hipGetLastError());
      if (it < a.max_iter) update(it);
    }
  } else {
    hipEvent_t ev[2];
    PFX_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
    PFX_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
    try {
      for (int it = 0; it <= a.max_iter; ++it) {
        hipLaunchKernelGGL(residual, dim3(B), dim3(ZB_THREADS), lds, s, d, a, it);
        PFX_HIP(hipGetLastError());
        PFX_HIP(hipMemcpyAsync(a.count_host + it, a.count + it, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        PFX_HIP(hipEventRecord(ev[it & 1], s));
        // Look one iteration back: once no scenario was active, nothing later can be.
        if (it > 0) {
          PFX_HIP(hipEventSynchronize(ev[(it - 1) & 1]));
          if (a.count_host[it - 1] == 0) break;
        }
        if (it == a.max_iter) break;
        update(it);
      }
    } catch (...) {
      (void)hipEventDestroy(ev[0]);
      (void)hipEventDestroy(ev[1]);
      throw;
    }
    PFX_HIP(hipEventDestroy(ev[0]));
    PFX_HIP(hipEventDestroy(ev[1]));
  }
  hipLaunchKernelGGL(zb_finish, dim3(B), dim3(ZB_THREADS), 0, s, d, a, net.slack_d.as<int>(),
                     net.vslack_d.as<double>());
  PFX_HIP(hipGetLastError());
}

template <typename T>
void zbus_step_t(DistNetwork& net, const ZbusLaunch& a, int iters, hipStream_t s) {
  const DistDev d = net.view();
  const T* W = sizeof(T) == 8 ? net.W64.as<T>() : net.W32.as<T>();
  const int B = a.batch;
  const int mt = (B + ZB_BM - 1) / ZB_BM;
  const int nt = net.Np / ZB_BN;
  const size_t lds = (size_t)d.nNs * 2 * sizeof(double);
  const int kb_need = (d.nNs + ZB_THREADS - 1) / ZB_THREADS;
  auto residual = kb_need <= 1 ? zb_residual<T, 1>
                  : kb_need <= 2 ? zb_residual<T, 2>
                  : kb_need <= 4 ? zb_residual<T, 4>
                  : kb_need <= 8 ? zb_residual<T, 8>
                                 : zb_residual<T, 16>;
  for (int k = 0; k < iters; ++k) {
    hipLaunchKernelGGL(residual, dim3(B), dim3(ZB_THREADS), lds, s, d, a, 0);
    PFX_HIP(hipGetLastError());
    if (a.sparse) {
      hipLaunchKernelGGL(zb_sparse<T>, dim3(B), dim3(WAVE), (size_t)d.nN * 2 * sizeof(T), s, d, a, 0);
    } else {
      launch_gemm<T>(d, W, a, 0, nt * mt, s);
    }
    PFX_HIP(hipGetLastError());
  }
}

}  // namespace

void zbus_init_slots(DistNetwork& net, const ZbusLaunch& a, hipStream_t s) {
  if (a.batch == 0) return;
  hipLaunchKernelGGL(zb_init, dim3(a.batch), dim3(ZB_THREADS), 0, s, net.view(), a);
  PFX_HIP(hipGetLastError());
}

void zbus_step(DistNetwork& net, bool mixed, const ZbusLaunch& a, int iters, hipStream_t s) {
  if (a.batch == 0) return;
  if (mixed) zbus_step_t<float>(net, a, iters, s);
  else zbus_step_t<double>(net, a, iters, s);
}

void zbus_finish_slots(DistNetwork& net, const ZbusLaunch& a, hipStream_t s) {
  if (a.batch == 0) return;
  hipLaunchKernelGGL(zb_finish, dim3(a.batch), dim3(ZB_THREADS), 0, s, net.view(), a, net.slack_d.as<int>(),
                     net.vslack_d.as<double>());
  PFX_HIP(hipGetLastError());
}

void run_zbus(DistNetwork& net, bool mixed, const ZbusLaunch& a, hipStream_t s) {
  if (a.batch == 0) return;
  if (mixed) run_zbus_t<float>(net, a, s);
  else run_zbus_t<double>(net, a, s);
}

}  // namespace pfx
