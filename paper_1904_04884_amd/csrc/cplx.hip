// Complex-valued object (absorption and phase).
//
// A complex plan holds the object as two real volumes of nz planes, the real
// parts and then the imaginary parts ([2][nz][ny][nx] FP32).  The hologram
// model and its adjoint need no kernels of their own: Re(IFFT2(FFT2(i y) H_j))
// is the real model with H_j multiplied by i, a carrier phase advanced by a
// quarter cycle, so the plan gives its second nz planes the carriers c_j + 1/4
// and the real kernels run on all 2 nz planes (their adjoint then returns the
// real and imaginary parts of A^T r).  What is complex is the regulariser
// (section "Methodology"): the l1 norm of Eq. (3) sums moduli, the TV of
// Eq. (4) takes the modulus of complex differences, and the soft threshold of
// Eq. (8) shrinks the modulus and keeps the phase.
//
// The TV prox is gradient projection on a complex dual, one complex value per
// direction, projected jointly on the unit ball of C^dims.  One step is two
// launches: u = v - tau D^T p into a scratch volume, then
// p <- (p + D u / (4 dims tau)) / max(1, |.|) in place (a voxel's new dual
// needs only its own dual and u at its forward neighbours).  The last launch
// forms u once more and writes the shrinkage of its modulus, with the
// occupancy flags of both parts.  These kernels stream whole volumes per step
// (no temporal blocking): the complex path is for parity and for
// complex-object work, not the benchmark's real path.
#include <hip/hip_runtime.h>

#include "rihvr_internal.h"

namespace rihvr {
namespace {

constexpr int kCThreads = 256;

struct CtvArgs {
  const float* v;        // input [2][nz][ny][nx]; nullptr: vol[st->prev]
  float* x;              // output; nullptr: vol[st->next]
  float* vol[3];
  const SolveState* st;
  float* u;              // scratch [2][nz][ny][nx]
  float* p[3];           // dual components [2][nz][ny][nx] each (p[2] unused in 2D)
  uint8_t* rowflag;      // nullable: [2 nz][ny], set where a row of a part is non-zero
  uint8_t* planeflag;    // [2 nz]
  int nx, ny, nz;        // nz: planes of one part
  int tv2;
  int first;             // the dual is zero (no step taken yet)
  float tau, c, thr;
};

__device__ __forceinline__ bool done(const SolveState* st) { return st != nullptr && st->done != 0; }

__device__ __forceinline__ const float* in_of(const CtvArgs& a) {
  return a.v != nullptr ? a.v : pick3<float>(a.vol[0], a.vol[1], a.vol[2], a.st->prev);
}
__device__ __forceinline__ float* out_of(const CtvArgs& a) {
  return a.x != nullptr ? a.x : pick3<float>(a.vol[0], a.vol[1], a.vol[2], a.st->next);
}

// -(D^T p) at voxel i of the part starting at offset o: the backward
// differences of the dual, zero where the forward difference is not defined.
__device__ __forceinline__ float neg_div(const CtvArgs& a, size_t i, size_t o, int x, int y, int z) {
  const size_t plane = (size_t)a.nx * a.ny;
  const float* px = a.p[0] + o;
  const float* py = a.p[1] + o;
  float d = (x + 1 < a.nx ? px[i] : 0.f) - (x > 0 ? px[i - 1] : 0.f);
  d += (y + 1 < a.ny ? py[i] : 0.f) - (y > 0 ? py[i - a.nx] : 0.f);
  if (!a.tv2) {
    const float* pz = a.p[2] + o;
    d += (z + 1 < a.nz ? pz[i] : 0.f) - (z > 0 ? pz[i - plane] : 0.f);
  }
  return d;
}

__global__ void __launch_bounds__(kCThreads) k_ctv_u(CtvArgs a) {
  if (done(a.st)) return;
  const size_t n = (size_t)a.nx * a.ny * a.nz;
  const float* __restrict__ v = in_of(a);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(i % a.nx), y = (int)((i / a.nx) % a.ny), z = (int)(i / ((size_t)a.nx * a.ny));
    for (int part = 0; part < 2; ++part) {
      const size_t o = part * n;
      a.u[o + i] = a.first ? v[o + i] : fmaf(a.tau, neg_div(a, i, o, x, y, z), v[o + i]);
    }
  }
}

__global__ void __launch_bounds__(kCThreads) k_ctv_p(CtvArgs a) {
  if (done(a.st)) return;
  const size_t n = (size_t)a.nx * a.ny * a.nz;
  const size_t plane = (size_t)a.nx * a.ny;
  const int nd = a.tv2 ? 2 : 3;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(i % a.nx), y = (int)((i / a.nx) % a.ny), z = (int)(i / plane);
    float q[3][2];
    float n2 = 0.f;
    for (int part = 0; part < 2; ++part) {
      const float* __restrict__ u = a.u + part * n;
      const float uc = u[i];
      const float g[3] = {x + 1 < a.nx ? u[i + 1] - uc : 0.f, y + 1 < a.ny ? u[i + a.nx] - uc : 0.f,
                          (!a.tv2 && z + 1 < a.nz) ? u[i + plane] - uc : 0.f};
      for (int d = 0; d < nd; ++d) {
        const float p0 = a.first ? 0.f : a.p[d][part * n + i];
        q[d][part] = fmaf(a.c, g[d], p0);
        n2 = fmaf(q[d][part], q[d][part], n2);
      }
    }
    const float inv = 1.f / fmaxf(1.f, sqrtf(n2));
    for (int d = 0; d < nd; ++d)
      for (int part = 0; part < 2; ++part) a.p[d][part * n + i] = q[d][part] * inv;
  }
}

// u once more, then the complex shrinkage (1 - thr/|u|)_+ u and the flags.
// In place is allowed (a voxel reads only its own v).
__global__ void __launch_bounds__(kCThreads) k_ctv_final(CtvArgs a) {
  if (done(a.st)) return;
  const size_t n = (size_t)a.nx * a.ny * a.nz;
  const float* v = in_of(a);
  float* xo = out_of(a);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(i % a.nx), y = (int)((i / a.nx) % a.ny), z = (int)(i / ((size_t)a.nx * a.ny));
    float ur = v[i], ui = v[n + i];
    if (!a.first) {
      ur = fmaf(a.tau, neg_div(a, i, 0, x, y, z), ur);
      ui = fmaf(a.tau, neg_div(a, i, n, x, y, z), ui);
    }
    const float mod = sqrtf(fmaf(ur, ur, ui * ui));
    float xr = 0.f, xi = 0.f;
    if (mod > a.thr) {
      const float s = 1.f - a.thr / mod;
      xr = s * ur;
      xi = s * ui;
    }
    xo[i] = xr;
    xo[n + i] = xi;
    if (a.rowflag != nullptr) {
      if (xr != 0.f) {
        a.rowflag[(size_t)z * a.ny + y] = 1;
        a.planeflag[z] = 1;
      }
      if (xi != 0.f) {
        a.rowflag[(size_t)(a.nz + z) * a.ny + y] = 1;
        a.planeflag[a.nz + z] = 1;
      }
    }
  }
}

// Per-block FP64 partials of sum |x| and of the complex TV of x (the solver's
// iterate x_it before the scalar kernel of its iteration, or x0 outside one).
struct CObjArgs {
  const float* x0; const float* x1; const float* x2;
  const SolveState* st;
  double* psum; double* ptv;
  int nx, ny, nz;        // nz: planes of one part
  int tv2;
};

__global__ void __launch_bounds__(kCThreads) k_cobj(CObjArgs a) {
  if (done(a.st)) return;
  __shared__ double red[2][kCThreads / 64];
  const float* __restrict__ xv = a.st != nullptr ? pick3<const float>(a.x0, a.x1, a.x2, a.st->it % 3) : a.x0;
  const size_t n = (size_t)a.nx * a.ny * a.nz;
  const size_t plane = (size_t)a.nx * a.ny;
  double s_acc = 0.0, t_acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const int x = (int)(i % a.nx), y = (int)((i / a.nx) % a.ny), z = (int)(i / plane);
    float g2 = 0.f, m2 = 0.f;
    for (int part = 0; part < 2; ++part) {
      const float* u = xv + part * n;
      const float c = u[i];
      m2 = fmaf(c, c, m2);
      const float gx = x + 1 < a.nx ? u[i + 1] - c : 0.f;
      const float gy = y + 1 < a.ny ? u[i + a.nx] - c : 0.f;
      const float gz = (!a.tv2 && z + 1 < a.nz) ? u[i + plane] - c : 0.f;
      g2 = fmaf(gx, gx, fmaf(gy, gy, fmaf(gz, gz, g2)));
    }
    s_acc += (double)sqrtf(m2);
    t_acc += (double)sqrtf(g2);
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
    for (int w = 0; w < kCThreads / 64; ++w) {
      s += red[0][w];
      t += red[1][w];
    }
    a.psum[blockIdx.x] = s;
    a.ptv[blockIdx.x] = t;
  }
}

int cgrid(size_t n) {
  const size_t b = (n + kCThreads - 1) / kCThreads;
  return (int)(b > 8192 ? 8192 : (b == 0 ? 1 : b));
}

}  // namespace

hipError_t launch_cprox(const ProxArgs& pa, hipStream_t s, int* launches) {
  CtvArgs a{};
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
  const dim3 g(cgrid((size_t)a.nx * a.ny * a.nz)), b(kCThreads);
  for (int k = 0; k < K; ++k) {
    a.first = k == 0 ? 1 : 0;
    hipLaunchKernelGGL(k_ctv_u, g, b, 0, s, a);
    hipLaunchKernelGGL(k_ctv_p, g, b, 0, s, a);
  }
  a.first = K == 0 ? 1 : 0;
  hipLaunchKernelGGL(k_ctv_final, g, b, 0, s, a);
  if (launches) *launches = 2 * K + 1;
  return hipGetLastError();
}

hipError_t launch_cobj(const ObjArgs& oa, int nblocks, hipStream_t s) {
  CObjArgs a{};
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
  hipLaunchKernelGGL(k_cobj, dim3(nblocks > 0 ? nblocks : 1), dim3(kCThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace rihvr
