// FP64 plans: the hologram model, its adjoint and the pieces of the FISTA
// iteration in double precision, for separating defects from FP32 rounding.
//
// The operator is the same angular-spectrum model (section "Methodology",
// Eq. 2 with the propagator A x = Re(sum_j IFFT2(FFT2(x_j) H_j))) from the
// same FP64 plan tables (theta, carriers), but computed plainly: complex
// transforms of whole planes (no packed half spectra), every plane's spectrum
// held at once, the filter cos(2 pi frac(z_j theta + c_j)) applied and summed
// over planes one frequency at a time.  The transforms are mixed-radix (2, 3)
// Stockham FFTs, one line per block, in LDS.  The FP32 path's kernels are
// specialised for FP32 register and LDS budgets; this path trades speed for a
// second implementation at 1e-9 of the FP64 oracle.
#include <hip/hip_runtime.h>

#include "rihvr_internal.h"

namespace rihvr {
namespace {

constexpr int kFThreads = 256;

__device__ __forceinline__ double2 cmul64(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}

// One transform of length N per block.  Line l starts at
// (l / lpg) * gstride + (l % lpg) * lstride; its elements are estride apart.
// Forward: exp(-2 pi i k n / N); inverse: exp(+...), both unscaled, then the
// result is multiplied by `scale`.  tw[k] = exp(-2 pi i k / N).
__global__ void __launch_bounds__(kFThreads) k64_fft(double2* data, int N, int lpg, size_t gstride, size_t lstride,
                                                      size_t estride, const double2* __restrict__ tw, int inverse,
                                                      double scale) {
  extern __shared__ double2 sh[];
  double2* a = sh;
  double2* b = sh + N;
  const int l = blockIdx.x;
  double2* base = data + (size_t)(l / lpg) * gstride + (size_t)(l % lpg) * lstride;
  for (int k = threadIdx.x; k < N; k += blockDim.x) a[k] = base[(size_t)k * estride];
  __syncthreads();
  const double sg = inverse ? 1.0 : -1.0;
  int ns = 1, rem = N;
  while (rem > 1) {
    const int R = (rem % 3 == 0) ? 3 : 2;
    rem /= R;
    const int tstep = N / (ns * R);
    for (int j = threadIdx.x; j < N / R; j += blockDim.x) {
      const int jm = j % ns;
      double2 v[3];
      for (int r = 0; r < R; ++r) {
        double2 w = tw[(jm * r * tstep) % N];
        if (inverse) w.y = -w.y;
        v[r] = cmul64(a[j + r * (N / R)], w);
      }
      double2 y[3];
      if (R == 2) {
        y[0] = make_double2(v[0].x + v[1].x, v[0].y + v[1].y);
        y[1] = make_double2(v[0].x - v[1].x, v[0].y - v[1].y);
      } else {
        // exp(sg 2 pi i / 3) = -1/2 + sg i sqrt(3)/2
        const double h = 0.86602540378443864676 * sg;
        const double2 s = make_double2(v[1].x + v[2].x, v[1].y + v[2].y);
        const double2 d = make_double2(v[1].x - v[2].x, v[1].y - v[2].y);
        y[0] = make_double2(v[0].x + s.x, v[0].y + s.y);
        const double2 m = make_double2(v[0].x - 0.5 * s.x, v[0].y - 0.5 * s.y);
        // +- i h d
        y[1] = make_double2(m.x - h * d.y, m.y + h * d.x);
        y[2] = make_double2(m.x + h * d.y, m.y - h * d.x);
      }
      const int idx = (j / ns) * ns * R + jm;
      for (int r = 0; r < R; ++r) b[idx + r * ns] = y[r];
    }
    __syncthreads();
    double2* t = a;
    a = b;
    b = t;
    ns *= R;
  }
  for (int k = threadIdx.x; k < N; k += blockDim.x) base[(size_t)k * estride] = make_double2(a[k].x * scale, a[k].y * scale);
}

__global__ void k64_to_complex(const double* __restrict__ x, double2* __restrict__ X, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    X[i] = make_double2(x[i], 0.0);
}

__global__ void k64_real(const double2* __restrict__ X, double* __restrict__ x, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    x[i] = X[i].x;
}

// cos(2 pi frac(z_j theta(f) + c_j)) at grid frequency (ky, kx): theta is
// tabulated for kx in [0, nx/2] (it depends on fx^2 only).
__device__ __forceinline__ double filt64(const Plan64Tables& t, int j, int ky, int kx) {
  const int kk = kx <= t.m ? kx : t.nx - kx;
  const double th = t.theta[(size_t)ky * (t.m + 1) + kk];
  const double2 zc = t.zc[j];
  double ph = fma(zc.x, th, zc.y);
  ph -= floor(ph);
  return cospi(2.0 * ph);
}

// S = sum_j X_j cos(phase_j), planes in order.
__global__ void k64_filter_sum(Plan64Tables t, const double2* __restrict__ X, double2* __restrict__ S) {
  const size_t np = (size_t)t.nx * t.ny;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += (size_t)gridDim.x * blockDim.x) {
    const int ky = (int)(i / t.nx), kx = (int)(i % t.nx);
    double2 acc = make_double2(0.0, 0.0);
    for (int j = 0; j < t.nzp; ++j) {
      const double c = filt64(t, j, ky, kx);
      const double2 v = X[(size_t)j * np + i];
      acc.x = fma(c, v.x, acc.x);
      acc.y = fma(c, v.y, acc.y);
    }
    S[i] = acc;
  }
}

// X_j = R cos(phase_j) for every plane.
__global__ void k64_filter_spread(Plan64Tables t, const double2* __restrict__ R, double2* __restrict__ X) {
  const size_t np = (size_t)t.nx * t.ny, n = np * t.nzp;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const size_t q = i % np;
    const int j = (int)(i / np), ky = (int)(q / t.nx), kx = (int)(q % t.nx);
    const double c = filt64(t, j, ky, kx);
    const double2 v = R[q];
    X[i] = make_double2(c * v.x, c * v.y);
  }
}

__global__ void k64_fill(double* out, double v, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) out[i] = v;
}

// out = a x + b y (element by element; out may alias x or y)
__global__ void k64_axpby(double* out, double a, const double* x, double b, const double* y, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    out[i] = fma(a, x[i], b * y[i]);
}

// per-block partial sums of (x - y)^2 over n elements, into part[blockIdx.x]
__global__ void __launch_bounds__(kFThreads) k64_sqdist(const double* x, const double* y, size_t n, double* part) {
  __shared__ double red[kFThreads / 64];
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const double d = x[i] - y[i];
    acc = fma(d, d, acc);
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kFThreads / 64; ++w) s += red[w];
    part[blockIdx.x] = s;
  }
}

int fgrid(size_t n) {
  const size_t b = (n + kFThreads - 1) / kFThreads;
  return (int)(b > 8192 ? 8192 : (b == 0 ? 1 : b));
}

// 2D transforms of `planes` planes of [ny][nx] complex values.
hipError_t fft2_64(const Plan64Tables& t, double2* X, int planes, bool inverse, hipStream_t s) {
  const size_t np = (size_t)t.nx * t.ny;
  const double sc = inverse ? 1.0 / (double)np : 1.0;
  // rows: nx points, ny * planes lines
  hipLaunchKernelGGL(k64_fft, dim3(t.ny * planes), dim3(kFThreads), 2 * t.nx * sizeof(double2), s, X, t.nx,
                     t.ny * planes, (size_t)0, (size_t)t.nx, (size_t)1, t.tw_x, inverse ? 1 : 0, 1.0);
  // columns: ny points nx apart, nx lines per plane
  hipLaunchKernelGGL(k64_fft, dim3(t.nx * planes), dim3(kFThreads), 2 * t.ny * sizeof(double2), s, X, t.ny, t.nx,
                     np, (size_t)1, (size_t)t.nx, t.tw_y, inverse ? 1 : 0, sc);
  return hipGetLastError();
}

}  // namespace

size_t f64_spectra_bytes(const Plan64Tables& t) {
  return (size_t)t.nx * t.ny * t.nzp * sizeof(double2);
}

hipError_t forward64(const Plan64Tables& t, const double* x, double* b, double2* X, double2* S, hipStream_t s) {
  const size_t np = (size_t)t.nx * t.ny, n = np * t.nzp;
  hipLaunchKernelGGL(k64_to_complex, dim3(fgrid(n)), dim3(kFThreads), 0, s, x, X, n);
  hipError_t e = fft2_64(t, X, t.nzp, false, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k64_filter_sum, dim3(fgrid(np)), dim3(kFThreads), 0, s, t, X, S);
  if ((e = fft2_64(t, S, 1, true, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k64_real, dim3(fgrid(np)), dim3(kFThreads), 0, s, S, b, np);
  return hipGetLastError();
}

hipError_t adjoint64(const Plan64Tables& t, const double* y, double* x, double2* X, double2* S, hipStream_t s) {
  const size_t np = (size_t)t.nx * t.ny, n = np * t.nzp;
  hipLaunchKernelGGL(k64_to_complex, dim3(fgrid(np)), dim3(kFThreads), 0, s, y, S, np);
  hipError_t e = fft2_64(t, S, 1, false, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k64_filter_spread, dim3(fgrid(n)), dim3(kFThreads), 0, s, t, S, X);
  if ((e = fft2_64(t, X, t.nzp, true, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k64_real, dim3(fgrid(n)), dim3(kFThreads), 0, s, X, x, n);
  return hipGetLastError();
}

hipError_t axpby64(double* out, double a, const double* x, double b, const double* y, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k64_axpby, dim3(fgrid(n)), dim3(kFThreads), 0, s, out, a, x, b, y, n);
  return hipGetLastError();
}

hipError_t fill64(double* out, double v, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k64_fill, dim3(fgrid(n)), dim3(kFThreads), 0, s, out, v, n);
  return hipGetLastError();
}

hipError_t sqdist64(const double* x, const double* y, size_t n, double* part, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(k64_sqdist, dim3(nblocks), dim3(kFThreads), 0, s, x, y, n, part);
  return hipGetLastError();
}

}  // namespace rihvr
