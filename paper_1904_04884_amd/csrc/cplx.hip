// Unfused gradient-projection TV prox and objective partials, templated on the
// element type T (float, double) and the number of parts NP (1: real object,
// 2: complex object).  They serve the complex object in FP32 and every FP64
// plan.
//
// Complex object.  A complex plan holds the object as two real volumes of nz
// planes, the real parts and then the imaginary parts ([2][nz][ny][nx]).  The
// hologram model and its adjoint need no kernels of their own:
// Re(IFFT2(FFT2(i y) H_j)) is the real model with H_j multiplied by i, a
// carrier phase advanced by a quarter cycle, so the plan gives its second nz
// planes the carriers c_j + 1/4 and the real kernels run on all 2 nz planes
// (their adjoint then returns the real and imaginary parts of A^T r).  What is
// complex is the regulariser (section "Methodology"): the l1 norm of Eq. (3)
// sums moduli, the TV of Eq. (4) takes the modulus of complex differences, and
// the soft threshold of Eq. (8) shrinks the modulus and keeps the phase.
//
// The TV prox is gradient projection on the dual, one value per part and
// direction, projected jointly on the unit ball.  One step is two launches:
// u = v - tau D^T p into a scratch volume, then p <- (p + D u / (4 dims tau)) /
// max(1, |.|) in place (a voxel's new dual needs only its own dual and u at its
// forward neighbours).  The last launch forms u once more and writes the
// threshold (real: max(u - thr, 0) or the signed form; complex: the shrinkage
// of the modulus), with the occupancy flags.  These kernels stream whole
// volumes per step (no temporal blocking): they are the complex-object and
// FP64 paths, not the benchmark's real FP32 path.
#include <hip/hip_runtime.h>

#include "rihvr_internal.h"

namespace rihvr {
namespace {

constexpr int kGThreads = 256;

template <class T>
struct GpArgs {
  const T* v;            // input [NP][nz][ny][nx]; nullptr: vol[st->prev]
  T* x;                  // output; nullptr: vol[st->next]
  T* vol[3];
  const SolveState* st;
  T* u;                  // scratch [NP][nz][ny][nx]
  T* p[3];               // dual components [NP][nz][ny][nx] each (p[2] unused in 2D)
  uint8_t* rowflag;      // nullable: [NP nz][ny], set where a row of a part is non-zero
  uint8_t* planeflag;    // [NP nz]
  int nx, ny, nz;        // nz: planes of one part
  int tv2;
  int nonneg;            // real object: x >= 0
  int first;             // the dual is zero (no step taken yet)
  T tau, c, thr;
};

__device__ __forceinline__ bool done(const SolveState* st) { return st != nullptr && st->done != 0; }

template <class T>
__device__ __forceinline__ const T* in_of(const GpArgs<T>& a) {
  return a.v != nullptr ? a.v : pick3<T>(a.vol[0], a.vol[1], a.vol[2], a.st->prev);
}
template <class T>
__device__ __forceinline__ T* out_of(const GpArgs<T>& a) {
  return a.x != nullptr ? a.x : pick3<T>(a.vol[0], a.vol[1], a.vol[2], a.st->next);
}

__device__ __forceinline__ float fmaT(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ float sqrtT(float a) { return sqrtf(a); }
__device__ __forceinline__ double sqrtT(double a) { return sqrt(a); }

// -(D^T p) at voxel i of the part starting at offset o: the backward
// differences of the dual, zero where the forward difference is not defined.
template <class T>
__device__ __forceinline__ T neg_div(const GpArgs<T>& a, size_t i, size_t o, int x, int y, int z) {
  const size_t plane = (size_t)a.nx * a.ny;
  const T* px = a.p[0] + o;
  const T* py = a.p[1] + o;
  T d = (x + 1 < a.nx ? px[i] : T(0)) - (x > 0 ? px[i - 1] : T(0));
  d += (y + 1 < a.ny ? py[i] : T(0)) - (y > 0 ? py[i - a.nx] : T(0));
  if (!a.tv2) {
    const T* pz = a.p[2] + o;
    d += (z + 1 < a.nz ? pz[i] : T(0)) - (z > 0 ? pz[i - plane] : T(0));
  }
  return d;
}

template <class T, int NP>
__global__ void __launch_bounds__(kGThreads) k_gp_u(GpArgs<T> a) {
  if (done(a.st)) return;
  const size_t n = (size_t)a.nx * a.ny * a.nz;
  const T* __restrict__ v = in_of(a);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(i % a.nx), y = (int)((i / a.nx) % a.ny), z = (int)(i / ((size_t)a.nx * a.ny));
#pragma unroll
    for (int part = 0; part < NP; ++part) {
      const size_t o = part * n;
      a.u[o + i] = a.first ? v[o + i] : fmaT(a.tau, neg_div(a, i, o, x, y, z), v[o + i]);
    }
  }
}

template <class T, int NP>
__global__ void __launch_bounds__(kGThreads) k_gp_p(GpArgs<T> a) {
  if (done(a.st)) return;
  const size_t n = (size_t)a.nx * a.ny * a.nz;
  const size_t plane = (size_t)a.nx * a.ny;
  const int nd = a.tv2 ? 2 : 3;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(i % a.nx), y = (int)((i / a.nx) % a.ny), z = (int)(i / plane);
    T q[3][NP];
    T n2 = T(0);
#pragma unroll
    for (int part = 0; part < NP; ++part) {
      const T* __restrict__ u = a.u + part * n;
      const T uc = u[i];
      const T g[3] = {x + 1 < a.nx ? u[i + 1] - uc : T(0), y + 1 < a.ny ? u[i + a.nx] - uc : T(0),
                      (!a.tv2 && z + 1 < a.nz) ? u[i + plane] - uc : T(0)};
      for (int d = 0; d < nd; ++d) {
        const T p0 = a.first ? T(0) : a.p[d][part * n + i];
        q[d][part] = fmaT(a.c, g[d], p0);
        n2 = fmaT(q[d][part], q[d][part], n2);
      }
    }
    const T s = n2 > T(1) ? sqrtT(n2) : T(1);
    for (int d = 0; d < nd; ++d)
#pragma unroll
      for (int part = 0; part < NP; ++part) a.p[d][part * n + i] = q[d][part] / s;
  }
}

// u once more, then the threshold and the flags.  In place is allowed (a
// voxel reads only its own v).
template <class T, int NP>
__global__ void __launch_bounds__(kGThreads) k_gp_final(GpArgs<T> a) {
  if (done(a.st)) return;
  const size_t n = (size_t)a.nx * a.ny * a.nz;
  const T* v = in_of(a);
  T* xo = out_of(a);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(i % a.nx), y = (int)((i / a.nx) % a.ny), z = (int)(i / ((size_t)a.nx * a.ny));
    T u[NP], r[NP];
    T m2 = T(0);
#pragma unroll
    for (int part = 0; part < NP; ++part) {
      u[part] = v[part * n + i];
      if (!a.first) u[part] = fmaT(a.tau, neg_div(a, i, part * n, x, y, z), u[part]);
      m2 = fmaT(u[part], u[part], m2);
    }
    if constexpr (NP == 1) {
      if (a.nonneg) {
        r[0] = u[0] - a.thr > T(0) ? u[0] - a.thr : T(0);
      } else {
        const T m = u[0] < T(0) ? -u[0] : u[0];
        r[0] = m > a.thr ? (u[0] < T(0) ? -(m - a.thr) : m - a.thr) : T(0);
      }
    } else {
      const T mod = sqrtT(m2);
      const T s = mod > a.thr ? T(1) - a.thr / mod : T(0);
#pragma unroll
      for (int part = 0; part < NP; ++part) r[part] = s * u[part];
    }
#pragma unroll
    for (int part = 0; part < NP; ++part) {
      xo[part * n + i] = r[part];
      if (a.rowflag != nullptr && r[part] != T(0)) {
        a.rowflag[(size_t)(part * a.nz + z) * a.ny + y] = 1;
        a.planeflag[part * a.nz + z] = 1;
      }
    }
  }
}

// Per-block FP64 partials of sum |x| and TV(x) (the solver's iterate x_it
// before the scalar kernel of its iteration, or x0 outside one).
template <class T>
struct ObjPartArgs {
  const T* x0; const T* x1; const T* x2;
  const SolveState* st;
  double* psum; double* ptv;
  int nx, ny, nz;        // nz: planes of one part
  int tv2;
};

template <class T, int NP>
__global__ void __launch_bounds__(kGThreads) k_gp_obj(ObjPartArgs<T> a) {
  if (done(a.st)) return;
  __shared__ double red[2][kGThreads / 64];
  const T* __restrict__ xv = a.st != nullptr ? pick3<const T>(a.x0, a.x1, a.x2, a.st->it % 3) : a.x0;
  const size_t n = (size_t)a.nx * a.ny * a.nz;
  const size_t plane = (size_t)a.nx * a.ny;
  double s_acc = 0.0, t_acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(i % a.nx), y = (int)((i / a.nx) % a.ny), z = (int)(i / plane);
    T g2 = T(0), m2 = T(0);
#pragma unroll
    for (int part = 0; part < NP; ++part) {
      const T* u = xv + part * n;
      const T c = u[i];
      m2 = fmaT(c, c, m2);
      const T gx = x + 1 < a.nx ? u[i + 1] - c : T(0);
      const T gy = y + 1 < a.ny ? u[i + a.nx] - c : T(0);
      const T gz = (!a.tv2 && z + 1 < a.nz) ? u[i + plane] - c : T(0);
      g2 = fmaT(gx, gx, fmaT(gy, gy, fmaT(gz, gz, g2)));
    }
    s_acc += (double)sqrtT(m2);
    t_acc += (double)sqrtT(g2);
  }
  for (int off = 32; off > 0; off >>= 1) {
    s_acc += __shfl_down(s_acc, off, 64);
    t_acc += __shfl_down(t_acc, off, 64);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wv] = s_acc;
    red[1][wv] = t_acc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0, t = 0.0;
    for (int w = 0; w < kGThreads / 64; ++w) {
      s += red[0][w];
      t += red[1][w];
    }
    a.psum[blockIdx.x] = s;
    a.ptv[blockIdx.x] = t;
  }
}

int ggrid(size_t n) {
  const size_t b = (n + kGThreads - 1) / kGThreads;
  return (int)(b > 8192 ? 8192 : (b == 0 ? 1 : b));
}

template <class T, int NP>
hipError_t run_gp(GpArgs<T> a, int K, hipStream_t s, int* launches) {
  const dim3 g(ggrid((size_t)a.nx * a.ny * a.nz)), b(kGThreads);
  for (int k = 0; k < K; ++k) {
    a.first = k == 0 ? 1 : 0;
    hipLaunchKernelGGL((k_gp_u<T, NP>), g, b, 0, s, a);
    hipLaunchKernelGGL((k_gp_p<T, NP>), g, b, 0, s, a);
  }
  a.first = K == 0 ? 1 : 0;
  hipLaunchKernelGGL((k_gp_final<T, NP>), g, b, 0, s, a);
  if (launches) *launches = 2 * K + 1;
  return hipGetLastError();
}

}  // namespace

hipError_t launch_cprox(const ProxArgs& pa, hipStream_t s, int* launches) {
  GpArgs<float> a{};
  a.v = pa.v;
  a.x = pa.x;
  for (int k = 0; k < 3; ++k) a.vol[k] = pa.vol[k];
  a.st = pa.st;
  a.u = pa.pb[0];
  for (int k = 0; k < 3; ++k) a.p[k] = pa.pa[k];
  a.rowflag = pa.rowflag;
  a.planeflag = pa.planeflag;
  a.nx = pa.nx;
  a.ny = pa.ny;
  a.nz = pa.nz / 2;
  a.tv2 = pa.tv2 ? 1 : 0;
  const double tau = pa.step * pa.tv;
  const int K = (tau > 0.0 && pa.inner_iters > 0) ? pa.inner_iters : 0;
  a.tau = (float)tau;
  a.c = K > 0 ? (float)(1.0 / ((a.tv2 ? 8.0 : 12.0) * tau)) : 0.f;
  a.thr = (float)(pa.step * pa.l1);
  return run_gp<float, 2>(a, K, s, launches);
}

hipError_t launch_cobj(const ObjArgs& oa, int nblocks, hipStream_t s) {
  ObjPartArgs<float> a{};
  a.x0 = oa.x0;
  a.x1 = oa.x1;
  a.x2 = oa.x2;
  a.st = oa.st;
  a.psum = oa.psum;
  a.ptv = oa.ptv;
  a.nx = oa.nx;
  a.ny = oa.ny;
  a.nz = oa.nz / 2;
  a.tv2 = oa.tv2;
  hipLaunchKernelGGL((k_gp_obj<float, 2>), dim3(nblocks > 0 ? nblocks : 1), dim3(kGThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_prox64(const Prox64Args& pa, hipStream_t s) {
  GpArgs<double> a{};
  a.v = pa.v;
  a.x = pa.x;
  a.u = pa.u;
  for (int k = 0; k < 3; ++k) a.p[k] = pa.p[k];
  a.nx = pa.nx;
  a.ny = pa.ny;
  a.nz = pa.nz;
  a.tv2 = pa.tv2;
  a.nonneg = pa.nonneg;
  const double tau = pa.step * pa.tv;
  const int K = (tau > 0.0 && pa.inner_iters > 0) ? pa.inner_iters : 0;
  a.tau = tau;
  a.c = K > 0 ? 1.0 / ((pa.tv2 ? 8.0 : 12.0) * tau) : 0.0;
  a.thr = pa.step * pa.l1;
  return pa.parts == 2 ? run_gp<double, 2>(a, K, s, nullptr) : run_gp<double, 1>(a, K, s, nullptr);
}

hipError_t launch_obj64(const double* x, int nx, int ny, int nz, int parts, int tv2, double* psum, double* ptv,
                        int nblocks, hipStream_t s) {
  ObjPartArgs<double> a{};
  a.x0 = a.x1 = a.x2 = x;
  a.psum = psum;
  a.ptv = ptv;
  a.nx = nx;
  a.ny = ny;
  a.nz = nz;
  a.tv2 = tv2;
  if (parts == 2) hipLaunchKernelGGL((k_gp_obj<double, 2>), dim3(nblocks), dim3(kGThreads), 0, s, a);
  else hipLaunchKernelGGL((k_gp_obj<double, 1>), dim3(nblocks), dim3(kGThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace rihvr
