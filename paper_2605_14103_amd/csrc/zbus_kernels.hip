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
//                 sparse Y_NN v, r, max |v * conj(r)|, flags, sum |v|
//   zb_gemm       D = R W (real-block form of Z r) on MFMA 16x16x4 tiles, with
//                 the FP64 update v += D fused into the epilogue
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "dist.hpp"

namespace pfx {

namespace {

constexpr int WAVE = 64;
constexpr int ZB_THREADS = 256;

__device__ __forceinline__ double nanmax(double a, double b) {
  if (a != a) return a;
  if (b != b) return b;
  return a > b ? a : b;
}

template <int BLOCK>
__device__ double block_nanmax(double v, double* red) {
  for (int off = WAVE / 2; off > 0; off >>= 1) v = nanmax(v, __shfl_xor(v, off, WAVE));
  if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = v;
  __syncthreads();
  double s = red[0];
  for (int i = 1; i < BLOCK / WAVE; ++i) s = nanmax(s, red[i]);
  __syncthreads();
  return s;
}

template <int BLOCK>
__device__ double block_sum(double v, double* red) {
  for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < BLOCK / WAVE; ++i) s += red[i];
  __syncthreads();
  return s;
}

// conj(s / v) for complex s, v given as (re, im)
__device__ __forceinline__ void conj_div(double sr, double si, double vr, double vi, double& outr,
                                         double& outi) {
  const double d = vr * vr + vi * vi;
  // s / v = s conj(v) / |v|^2
  const double qr = (sr * vr + si * vi) / d;
  const double qi = (si * vr - sr * vi) / d;
  outr = qr;
  outi = -qi;
}

__global__ __launch_bounds__(ZB_THREADS) void zb_init(DistDev net, ZbusLaunch a) {
  const int b = blockIdx.x;
  double* v = a.v + (int64_t)b * net.Kp;
  for (int i = threadIdx.x; i < 2 * net.nN; i += ZB_THREADS) v[i] = net.v0[i];
  if (threadIdx.x == 0) {
    a.active[b] = 1;
    a.iters[b] = 0;
    a.converged[b] = 0;
    a.st[3 * b + 0] = 0.0;
    a.st[3 * b + 1] = 0.0;
    a.st[3 * b + 2] = 0.0;
  }
}

template <typename T>
__global__ __launch_bounds__(ZB_THREADS) void zb_residual(DistDev net, ZbusLaunch a, int it) {
  extern __shared__ double vs[];  // [2 nN]
  __shared__ double red[ZB_THREADS / WAVE];
  const int b = blockIdx.x;
  if (a.active[b] == 0) return;
  const int nN = net.nN;
  const double* v = a.v + (int64_t)b * net.Kp;
  for (int i = threadIdx.x; i < 2 * nN; i += ZB_THREADS) vs[i] = v[i];
  __syncthreads();
  const double* SW = a.s_wye + 2 * (int64_t)b * a.ld;
  const double* SD = a.s_delta + 2 * (int64_t)b * a.ld;
  T* r = reinterpret_cast<T*>(a.r) + (int64_t)b * net.Kp;
  double mm = 0.0, sabs = 0.0;
  for (int i = threadIdx.x; i < nN; i += ZB_THREADS) {
    const double vr = vs[2 * i], vi = vs[2 * i + 1];
    double ir = 0.0, ii = 0.0;
    if (net.wye[i]) {  // wye: -conj(S / v)
      const int e = net.free2ext[i];
      double cr, ci;
      conj_div(SW[2 * e], SW[2 * e + 1], vr, vi, cr, ci);
      ir -= cr;
      ii -= ci;
    }
    const int nx = net.d_next[i];
    if (nx >= 0) {  // delta: branch x->next carries S_x, branch prev->x carries S_prev
      const int pv = net.d_prev[i];
      const int e = net.free2ext[i], ep = net.free2ext[pv];
      double axr, axi, apr, api;
      conj_div(SD[2 * e], SD[2 * e + 1], vr - vs[2 * nx], vi - vs[2 * nx + 1], axr, axi);
      conj_div(SD[2 * ep], SD[2 * ep + 1], vs[2 * pv] - vr, vs[2 * pv + 1] - vi, apr, api);
      ir -= axr - apr;
      ii -= axi - api;
    }
    double yr = net.c[2 * i], yi = net.c[2 * i + 1];
    for (int p = net.y_ptr[i]; p < net.y_ptr[i + 1]; ++p) {
      const int j = net.y_col[p];
      const double gr = net.y_re[p], gi = net.y_im[p];
      const double xr = vs[2 * j], xi = vs[2 * j + 1];
      yr += gr * xr - gi * xi;
      yi += gr * xi + gi * xr;
    }
    const double rr = ir - yr, ri = ii - yi;
    // v * conj(r)
    const double dr = vr * rr + vi * ri, di = vi * rr - vr * ri;
    mm = nanmax(mm, sqrt(dr * dr + di * di));
    sabs += sqrt(vr * vr + vi * vi);
    r[2 * i] = (T)rr;
    r[2 * i + 1] = (T)ri;
  }
  mm = block_nanmax<ZB_THREADS>(mm, red);
  sabs = block_sum<ZB_THREADS>(sabs, red);
  if (threadIdx.x == 0) {
    double* st = a.st + 3 * (int64_t)b;
    st[0] = mm;
    if (it > 0) st[2] = fabs(sabs - st[1]);
    st[1] = sabs;
    if (mm <= a.tol) {
      a.converged[b] = 1;
      a.active[b] = 0;
    } else if (!(mm == mm) || it >= a.max_iter) {
      a.active[b] = 0;
    } else {
      a.iters[b] = it + 1;
      atomicAdd(&a.count[it], 1);
    }
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

// D = R W on a ZB_BM x ZB_BN tile per workgroup (4 waves, 2 x 2, 64 x 64 each,
// 4 x 4 MFMA 16x16x4 tiles per wave), K in steps of ZB_BK staged through LDS,
// double buffered.  Epilogue: v += D for active scenarios (FP64).
template <typename T>
__global__ __launch_bounds__(256) void zb_gemm(DistDev net, const T* __restrict__ W, ZbusLaunch a) {
  using V4 = typename Mfma<T>::V4;
  __shared__ T As[2][ZB_BK][ZB_BM];
  __shared__ T Bs[2][ZB_BK][ZB_BN];
  const int tile_n = blockIdx.x, tile_m = blockIdx.y;
  const int row0 = tile_m * ZB_BM, col0 = tile_n * ZB_BN;
  const int t = threadIdx.x;
  {
    int act = 0;
    if (t < ZB_BM && row0 + t < a.batch) act = a.active[row0 + t];
    if (!__syncthreads_or(act)) return;
  }
  const int Kp = net.Kp, Np = net.Np;
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

  T ra[8], rb[8];
  auto gload = [&](int kt) {
#pragma unroll
    for (int q = 0; q < 8; ++q) ra[q] = Ag[kt * ZB_BK + q];
#pragma unroll
    for (int q = 0; q < 8; ++q) rb[q] = Bg[(int64_t)kt * ZB_BK * Np + q];
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 8; ++q) As[buf][ac + q][ar] = ra[q];
#pragma unroll
    for (int q = 0; q < 8; ++q) Bs[buf][br][bc + q] = rb[q];
  };
  const int nk = Kp / ZB_BK;
  gload(0);
  sstore(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) gload(kt + 1);
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
    if (kt + 1 < nk) sstore(buf ^ 1);
    __syncthreads();
  }
  const int ncol = 2 * net.nN;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int vv = 0; vv < 4; ++vv) {
      const int row = row0 + wm * 64 + i * 16 + Mfma<T>::out_row(lane, vv);
      if (row >= a.batch || a.active[row] == 0) continue;
      double* vrow = a.v + (int64_t)row * Kp;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int col = col0 + wn * 64 + j * 16 + (lane & 15);
        if (col < ncol) vrow[col] += (double)acc[i][j][vv];
      }
    }
  }
}

__global__ __launch_bounds__(ZB_THREADS) void zb_finish(DistDev net, ZbusLaunch a, const int* slack,
                                                       const double* vslack) {
  const int b = blockIdx.x;
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

template <typename T>
void run_zbus_t(DistNetwork& net, const ZbusLaunch& a, hipStream_t s) {
  const DistDev d = net.view();
  const T* W = sizeof(T) == 8 ? net.W64.as<T>() : net.W32.as<T>();
  const int B = a.batch;
  const int mt = (B + ZB_BM - 1) / ZB_BM;
  const int nt = net.Np / ZB_BN;
  const size_t lds = 2 * (size_t)net.nN * sizeof(double);
  hipLaunchKernelGGL(zb_init, dim3(B), dim3(ZB_THREADS), 0, s, d, a);
  PFX_HIP(hipGetLastError());
  PFX_HIP(hipMemsetAsync(a.count, 0, sizeof(int32_t) * (a.max_iter + 1), s));
  hipEvent_t ev[2];
  PFX_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
  PFX_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
  try {
    for (int it = 0; it <= a.max_iter; ++it) {
      hipLaunchKernelGGL(zb_residual<T>, dim3(B), dim3(ZB_THREADS), lds, s, d, a, it);
      PFX_HIP(hipGetLastError());
      PFX_HIP(hipMemcpyAsync(a.count_host + it, a.count + it, sizeof(int32_t), hipMemcpyDeviceToHost, s));
      PFX_HIP(hipEventRecord(ev[it & 1], s));
      // Look one iteration back: once no scenario was active, nothing later can be.
      if (it > 0) {
        PFX_HIP(hipEventSynchronize(ev[(it - 1) & 1]));
        if (a.count_host[it - 1] == 0) break;
      }
      if (it == a.max_iter) break;
      hipLaunchKernelGGL(zb_gemm<T>, dim3(nt, mt), dim3(256), 0, s, d, W, a);
      PFX_HIP(hipGetLastError());
    }
  } catch (...) {
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    throw;
  }
  PFX_HIP(hipEventDestroy(ev[0]));
  PFX_HIP(hipEventDestroy(ev[1]));
  hipLaunchKernelGGL(zb_finish, dim3(B), dim3(ZB_THREADS), 0, s, d, a, net.slack_d.as<int>(),
                     net.vslack_d.as<double>());
  PFX_HIP(hipGetLastError());
}

}  // namespace

void run_zbus(DistNetwork& net, bool mixed, const ZbusLaunch& a, hipStream_t s) {
  if (a.batch == 0) return;
  if (mixed) run_zbus_t<float>(net, a, s);
  else run_zbus_t<double>(net, a, s);
}

}  // namespace pfx
