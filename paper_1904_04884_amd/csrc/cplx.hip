// Gradient-projection TV prox (one step per launch) and objective partials, templated on the
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
// direction, projected jointly on the unit ball.  One launch takes one step,
// streamed along z with the dual staged in LDS and u formed once per voxel,
// and writes the other of two dual sets, so the sets alternate step by step.
// The last launch forms u once more and writes the threshold (real: max(u -
// thr, 0) or the signed form; complex: the shrinkage of the modulus), with the
// occupancy flags.  A step streams v, one dual set in and the other out (56 B
// per complex voxel, plus the tile halo); there is no temporal blocking: these
// kernels are the complex-object and FP64 paths, not the benchmark's real
// FP32 path.
#include <hip/hip_runtime.h>

#include <utility>

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
  T* p[3];               // dual read by a step and by the final launch, [NP][nz][ny][nx] each
                         // (p[2] unused in 2D)
  T* q[3];               // dual written by a step (the two sets alternate)
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

// One gradient-projection step, streamed along z.  A block of 512 threads
// owns a 64 x 8 tile of every plane and walks the planes upward (a 64 x 16
// tile in FP32, two rows per thread, measured 3% slower: half the blocks fit
// a CU by LDS).  For each plane it stages in LDS the dual it needs (p_x with
// its -x halo column, p_y with its -y halo row, p_z of this plane and of the
// one below, all on the tile and its +x / +y halo), forms u = v - tau D^T p
// once per voxel of the tile and its halo, and then writes the new dual of the
// plane below, q = p + c D u, p' = q / max(1, |q|), from u at the voxel and
// its +x, +y and +z neighbours.  The loads of a plane (its dual stage and v)
// go to registers two planes ahead and into LDS when the plane's turn comes,
// so they are in flight while the plane before is computed (132 -> 87 ms per
// outer iteration at 1024^2 x 256 complex).  It reads the dual set a.p and
// writes the other set a.q.  FP32 runs it only for an odd last step
// (k_gp_zstep2 takes the steps in pairs); FP64 runs every step with it.
constexpr int kZX = 64, kZT = 512;
template <class T>
constexpr int zstep_rows() { return 8; }

template <class T, int NP>
__global__ void __launch_bounds__(kZT) k_gp_zstep(GpArgs<T> a) {
  if (done(a.st)) return;
  constexpr int NT = kZT, kZY = zstep_rows<T>(), RY = kZY / (kZT / kZX);   // rows of the tile, per thread
  constexpr int UW = kZX + 1, UH = kZY + 1, UA = UW * UH;      // u and p_z: tile + forward halo
  constexpr int XW = kZX + 2, XA = XW * UH;                      // p_x: also the -x column
  constexpr int YA = UW * (kZY + 2);                             // p_y: also the -y row
  __shared__ T us[2][NP][UA];
  __shared__ T pxs[NP][XA];
  __shared__ T pys[NP][YA];
  __shared__ T pzs[2][NP][UA];
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const size_t plane = (size_t)nx * ny, n = plane * nz;
  const int tx = threadIdx.x % kZX, ty0 = threadIdx.x / kZX;   // rows ty0 + r * (kZT / kZX)
  const int x0 = blockIdx.x * kZX, y0 = blockIdx.y * kZY;
  const int x = x0 + tx;
  const bool tv3 = !a.tv2;
  const bool pre = !a.first;   // the dual is read (zero on the first step)
  const T* __restrict__ v = in_of(a);
  // What a thread loads of plane z: its points of the p_x, p_y and p_z stages
  // (tile and halo, as laid out in LDS) and of v on the u region, held in
  // registers so that plane z + 2 is in flight while plane z is computed.
  constexpr int NXR = (XA + NT - 1) / NT, NYR = (YA + NT - 1) / NT, NUR = (UA + NT - 1) / NT;
  struct Plane {
    T px[NXR][NP], py[NYR][NP], pz[NUR][NP], v[NUR][NP];
  };
  auto fetch = [&](int z, Plane& r) {
    const size_t base = (size_t)z * plane;
#pragma unroll
    for (int i = 0; i < NXR; ++i) {
      const int k = threadIdx.x + i * NT, xx = x0 - 1 + k % XW, yy = y0 + k / XW;
      const bool ok = pre && k < XA && xx >= 0 && xx < nx && yy < ny;
#pragma unroll
      for (int part = 0; part < NP; ++part)
        r.px[i][part] = ok ? a.p[0][part * n + base + (size_t)yy * nx + xx] : T(0);
    }
#pragma unroll
    for (int i = 0; i < NYR; ++i) {
      const int k = threadIdx.x + i * NT, xx = x0 + k % UW, yy = y0 - 1 + k / UW;
      const bool ok = pre && k < YA && xx < nx && yy >= 0 && yy < ny;
#pragma unroll
      for (int part = 0; part < NP; ++part)
        r.py[i][part] = ok ? a.p[1][part * n + base + (size_t)yy * nx + xx] : T(0);
    }
#pragma unroll
    for (int i = 0; i < NUR; ++i) {
      const int k = threadIdx.x + i * NT, xx = x0 + k % UW, yy = y0 + k / UW;
      const bool ok = k < UA && xx < nx && yy < ny;
      const size_t o = base + (size_t)yy * nx + xx;
#pragma unroll
      for (int part = 0; part < NP; ++part) {
        r.pz[i][part] = (ok && pre && tv3) ? a.p[2][part * n + o] : T(0);
        r.v[i][part] = ok ? v[part * n + o] : T(0);
      }
    }
  };
  // the dual of plane z into LDS (p_z into parity slot z & 1)
  auto commit = [&](int z, const Plane& r) {
    if (!pre) return;
#pragma unroll
    for (int i = 0; i < NXR; ++i) {
      const int k = threadIdx.x + i * NT;
      if (k < XA)
#pragma unroll
        for (int part = 0; part < NP; ++part) pxs[part][k] = r.px[i][part];
    }
#pragma unroll
    for (int i = 0; i < NYR; ++i) {
      const int k = threadIdx.x + i * NT;
      if (k < YA)
#pragma unroll
        for (int part = 0; part < NP; ++part) pys[part][k] = r.py[i][part];
    }
    if (tv3) {
#pragma unroll
      for (int i = 0; i < NUR; ++i) {
        const int k = threadIdx.x + i * NT;
        if (k < UA)
#pragma unroll
          for (int part = 0; part < NP; ++part) pzs[z & 1][part][k] = r.pz[i][part];
      }
    }
  };
  // u of plane z on the tile and its forward halo into slot z & 1 (v from the
  // registers, the dual from LDS)
  auto form_u = [&](int z, const Plane& r) {
#pragma unroll
    for (int i = 0; i < NUR; ++i) {
      const int k = threadIdx.x + i * NT;
      if (k >= UA) continue;
      const int lx = k % UW, ly = k / UW, xx = x0 + lx, yy = y0 + ly;
      const bool ok = xx < nx && yy < ny;
#pragma unroll
      for (int part = 0; part < NP; ++part) {
        T u = r.v[i][part];
        if (ok && pre) {
          T d = (xx + 1 < nx ? pxs[part][ly * XW + lx + 1] : T(0)) - (xx > 0 ? pxs[part][ly * XW + lx] : T(0));
          d += (yy + 1 < ny ? pys[part][(ly + 1) * UW + lx] : T(0)) - (yy > 0 ? pys[part][ly * UW + lx] : T(0));
          if (tv3)
            d += (z + 1 < nz ? pzs[z & 1][part][k] : T(0)) - (z > 0 ? pzs[(z & 1) ^ 1][part][k] : T(0));
          u = fmaT(a.tau, d, u);
        }
        us[z & 1][part][k] = u;
      }
    }
  };
  Plane R;
  fetch(0, R);
  commit(0, R);
  __syncthreads();
  form_u(0, R);
  if (nz > 1) fetch(1, R);
  for (int z = 0; z < nz; ++z) {
    const int s0 = z & 1, s1 = s0 ^ 1;
    // this thread's dual of plane z, read before plane z + 1 is staged over it
    T p0[RY][3][NP];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const int ty = ty0 + r * (kZT / kZX), ko = ty * UW + tx;
#pragma unroll
      for (int part = 0; part < NP; ++part) {
        p0[r][0][part] = pre ? pxs[part][ty * XW + tx + 1] : T(0);
        p0[r][1][part] = pre ? pys[part][(ty + 1) * UW + tx] : T(0);
        p0[r][2][part] = (pre && tv3) ? pzs[s0][part][ko] : T(0);
      }
    }
    __syncthreads();
    if (z + 1 < nz) {
      commit(z + 1, R);
      __syncthreads();
      form_u(z + 1, R);
      if (z + 2 < nz) fetch(z + 2, R);   // in flight while plane z is computed
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const int ty = ty0 + r * (kZT / kZX), ko = ty * UW + tx, y = y0 + ty;
      if (x < nx && y < ny) {
        const size_t i = (size_t)z * plane + (size_t)y * nx + x;
        const bool hx = x + 1 < nx, hy = y + 1 < ny, hz = tv3 && z + 1 < nz;
        const int nd = tv3 ? 3 : 2;
        T q[3][NP];
        T n2 = T(0);
#pragma unroll
        for (int part = 0; part < NP; ++part) {
          const T uc = us[s0][part][ko];
          const T g[3] = {hx ? us[s0][part][ko + 1] - uc : T(0), hy ? us[s0][part][ko + UW] - uc : T(0),
                          hz ? us[s1][part][ko] - uc : T(0)};
          for (int d = 0; d < nd; ++d) {
            q[d][part] = fmaT(a.c, g[d], p0[r][d][part]);
            n2 = fmaT(q[d][part], q[d][part], n2);
          }
        }
        const T sc = n2 > T(1) ? sqrtT(n2) : T(1);
        for (int d = 0; d < nd; ++d)
#pragma unroll
          for (int part = 0; part < NP; ++part) a.q[d][part * n + i] = q[d][part] / sc;
      }
    }
  }
}

// Two gradient-projection steps in one launch, streamed along z like
// k_gp_zstep: the first step's dual p' never leaves LDS, so a pair of steps
// reads p and v once and writes p'' once (56 B per complex voxel per two
// steps instead of per step).  The second step needs p' on the tile and a
// one-voxel ring around it, which needs u on the tile and a ring of two on the
// +x / +y side and one on the other sides, which needs p on a ring of two on
// the -x / -y side.  Regions, relative to the tile origin:
//   p_x staged  x in [-2, 65], y in [-1, 9]     u, v, p_z   x in [-1, 65], y in [-1, 9]
//   p_y staged  x in [-1, 65], y in [-2, 9]     p'          x in [-1, 64], y in [-1, 8]
//   u' = v - tau D^T p'   x in [0, 64], y in [0, 8]          p''   the 64 x 8 tile
// At plane z the block stages p(z + 1), forms u(z + 1), steps p'(z), forms
// u'(z) and steps p''(z - 1), with every plane's loads issued into registers
// two planes ahead.  FP32 only (its LDS, 78 KB, holds two blocks per CU):
// 87 -> 69 ms per outer iteration at 1024^2 x 256 complex.
template <class T, int NP>
__global__ void __launch_bounds__(kZT) k_gp_zstep2(GpArgs<T> a) {
  if (done(a.st)) return;
  constexpr int NT = kZT, TW = kZX, TH = kZT / kZX;
  constexpr int AW = TW + 3, AH = TH + 3, AA = AW * AH;    // u, v, p_z
  constexpr int XW = TW + 4, XA = XW * AH;                 // p_x
  constexpr int YW = AW, YH = TH + 4, YA = YW * YH;        // p_y
  constexpr int BW = TW + 2, BH = TH + 2, BA = BW * BH;    // p'
  constexpr int CW = TW + 1, CH = TH + 1, CA = CW * CH;    // u'
  __shared__ T pxs[NP][XA];
  __shared__ T pys[NP][YA];
  __shared__ T pzs[2][NP][AA];
  __shared__ T vs[2][NP][AA];
  __shared__ T us[2][NP][AA];
  __shared__ T qxs[NP][BA];
  __shared__ T qys[NP][BA];
  __shared__ T qzs[2][NP][BA];
  __shared__ T ws[2][NP][CA];
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const size_t plane = (size_t)nx * ny, n = plane * nz;
  const int x0 = blockIdx.x * TW, y0 = blockIdx.y * TH;
  const bool tv3 = !a.tv2;
  const bool pre = !a.first;   // p is read (zero before the first step)
  const T tau = a.tau, cc = a.c;
  const T* __restrict__ v = in_of(a);
  auto inside = [&](int gx, int gy) { return gx >= 0 && gx < nx && gy >= 0 && gy < ny; };
  // a plane's loads, in registers until its turn
  constexpr int NXR = (XA + NT - 1) / NT, NYR = (YA + NT - 1) / NT, NAR = (AA + NT - 1) / NT;
  struct Plane {
    T px[NXR][NP], py[NYR][NP], pz[NAR][NP], v[NAR][NP];
  };
  auto fetch = [&](int z, Plane& r) {
    const size_t base = (size_t)z * plane;
#pragma unroll
    for (int i = 0; i < NXR; ++i) {
      const int k = threadIdx.x + i * NT, gx = x0 + k % XW - 2, gy = y0 + k / XW - 1;
      const bool ok = pre && k < XA && inside(gx, gy);
#pragma unroll
      for (int part = 0; part < NP; ++part)
        r.px[i][part] = ok ? a.p[0][part * n + base + (size_t)gy * nx + gx] : T(0);
    }
#pragma unroll
    for (int i = 0; i < NYR; ++i) {
      const int k = threadIdx.x + i * NT, gx = x0 + k % YW - 1, gy = y0 + k / YW - 2;
      const bool ok = pre && k < YA && inside(gx, gy);
#pragma unroll
      for (int part = 0; part < NP; ++part)
        r.py[i][part] = ok ? a.p[1][part * n + base + (size_t)gy * nx + gx] : T(0);
    }
#pragma unroll
    for (int i = 0; i < NAR; ++i) {
      const int k = threadIdx.x + i * NT, gx = x0 + k % AW - 1, gy = y0 + k / AW - 1;
      const bool ok = k < AA && inside(gx, gy);
      const size_t o = base + (size_t)(ok ? gy : 0) * nx + (ok ? gx : 0);
#pragma unroll
      for (int part = 0; part < NP; ++part) {
        r.pz[i][part] = (ok && pre && tv3) ? a.p[2][part * n + o] : T(0);
        r.v[i][part] = ok ? v[part * n + o] : T(0);
      }
    }
  };
  auto commit = [&](int z, const Plane& r) {
    const int sl = z & 1;
#pragma unroll
    for (int i = 0; i < NXR; ++i) {
      const int k = threadIdx.x + i * NT;
      if (k < XA)
#pragma unroll
        for (int part = 0; part < NP; ++part) pxs[part][k] = r.px[i][part];
    }
#pragma unroll
    for (int i = 0; i < NYR; ++i) {
      const int k = threadIdx.x + i * NT;
      if (k < YA)
#pragma unroll
        for (int part = 0; part < NP; ++part) pys[part][k] = r.py[i][part];
    }
#pragma unroll
    for (int i = 0; i < NAR; ++i) {
      const int k = threadIdx.x + i * NT;
      if (k < AA)
#pragma unroll
        for (int part = 0; part < NP; ++part) {
          pzs[sl][part][k] = r.pz[i][part];
          vs[sl][part][k] = r.v[i][part];
        }
    }
  };
  // u(z) = v - tau D^T p on the u region
  auto form_u = [&](int z) {
    const int sl = z & 1;
#pragma unroll
    for (int i = 0; i < NAR; ++i) {
      const int k = threadIdx.x + i * NT;
      if (k >= AA) continue;
      const int lx = k % AW - 1, ly = k / AW - 1, gx = x0 + lx, gy = y0 + ly;
      const bool in = inside(gx, gy);
#pragma unroll
      for (int part = 0; part < NP; ++part) {
        T u = vs[sl][part][k];
        if (in && pre) {
          const int ix = (ly + 1) * XW + lx + 2, iy = (ly + 2) * YW + lx + 1;
          T d = (gx + 1 < nx ? pxs[part][ix] : T(0)) - (gx > 0 ? pxs[part][ix - 1] : T(0));
          d += (gy + 1 < ny ? pys[part][iy] : T(0)) - (gy > 0 ? pys[part][iy - YW] : T(0));
          if (tv3) d += (z + 1 < nz ? pzs[sl][part][k] : T(0)) - (z > 0 ? pzs[sl ^ 1][part][k] : T(0));
          u = fmaT(tau, d, u);
        }
        us[sl][part][k] = in ? u : T(0);
      }
    }
  };
  constexpr int NBR = (BA + NT - 1) / NT, NCR = (CA + NT - 1) / NT;
  Plane R;
  fetch(0, R);
  commit(0, R);
  __syncthreads();
  form_u(0);
  if (nz > 1) fetch(1, R);
  // this thread's p' of the plane below on the tile (second step's input)
  const int tx = threadIdx.x % TW, ty = threadIdx.x / TW, gxt = x0 + tx, gyt = y0 + ty;
  const bool int_ = inside(gxt, gyt);
  T pp1[3][NP];
  // p''(m) on the tile from u'(m) (slot m & 1), u'(m + 1) (the other slot, when
  // hz) and pp1 = p'(m); stored to a.q
  auto step2_out = [&](int m, bool hz) {
    const int sl = m & 1;
    const int kc = ty * CW + tx;
    T q[3][NP];
    T n2 = T(0);
#pragma unroll
    for (int part = 0; part < NP; ++part) {
      const T wc = ws[sl][part][kc];
      const T g[3] = {gxt + 1 < nx ? ws[sl][part][kc + 1] - wc : T(0), gyt + 1 < ny ? ws[sl][part][kc + CW] - wc : T(0),
                      hz ? ws[sl ^ 1][part][kc] - wc : T(0)};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        q[d][part] = (d < 2 || tv3) ? fmaT(cc, g[d], pp1[d][part]) : T(0);
        n2 = fmaT(q[d][part], q[d][part], n2);
      }
    }
    if (int_) {
      const T sc = n2 > T(1) ? sqrtT(n2) : T(1);
      const size_t i = (size_t)m * plane + (size_t)gyt * nx + gxt;
      const int nd = tv3 ? 3 : 2;
      for (int d = 0; d < nd; ++d)
#pragma unroll
        for (int part = 0; part < NP; ++part) a.q[d][part * n + i] = q[d][part] / sc;
    }
  };
  for (int z = 0; z < nz; ++z) {
    const int sl = z & 1;
    // p(z) on the p' region, read before plane z + 1 is staged over it
    T p0[NBR][3][NP];
#pragma unroll
    for (int i = 0; i < NBR; ++i) {
      const int k = threadIdx.x + i * NT, lx = k % BW - 1, ly = k / BW - 1;
      const bool ok = pre && k < BA;
#pragma unroll
      for (int part = 0; part < NP; ++part) {
        p0[i][0][part] = ok ? pxs[part][(ly + 1) * XW + lx + 2] : T(0);
        p0[i][1][part] = ok ? pys[part][(ly + 2) * YW + lx + 1] : T(0);
        p0[i][2][part] = (ok && tv3) ? pzs[sl][part][(ly + 1) * AW + lx + 1] : T(0);
      }
    }
    __syncthreads();
    if (z + 1 < nz) {
      commit(z + 1, R);
      __syncthreads();
      form_u(z + 1);
      if (z + 2 < nz) fetch(z + 2, R);   // in flight while this plane is computed
    }
    __syncthreads();
    // first step: p'(z) on the p' region
    const bool hz1 = tv3 && z + 1 < nz;
#pragma unroll
    for (int i = 0; i < NBR; ++i) {
      const int k = threadIdx.x + i * NT;
      if (k >= BA) continue;
      const int lx = k % BW - 1, ly = k / BW - 1, gx = x0 + lx, gy = y0 + ly;
      const int ku = (ly + 1) * AW + lx + 1;
      T q[3][NP];
      T n2 = T(0);
#pragma unroll
      for (int part = 0; part < NP; ++part) {
        const T uc = us[sl][part][ku];
        const T g[3] = {gx + 1 < nx ? us[sl][part][ku + 1] - uc : T(0), gy + 1 < ny ? us[sl][part][ku + AW] - uc : T(0),
                        hz1 ? us[sl ^ 1][part][ku] - uc : T(0)};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          q[d][part] = (d < 2 || tv3) ? fmaT(cc, g[d], p0[i][d][part]) : T(0);
          n2 = fmaT(q[d][part], q[d][part], n2);
        }
      }
      const bool in = inside(gx, gy);
      const T sc = n2 > T(1) ? sqrtT(n2) : T(1);
#pragma unroll
      for (int part = 0; part < NP; ++part) {
        qxs[part][k] = in ? q[0][part] / sc : T(0);
        qys[part][k] = in ? q[1][part] / sc : T(0);
        qzs[sl][part][k] = in ? q[2][part] / sc : T(0);
      }
    }
    __syncthreads();
    // u'(z) = v - tau D^T p' on the u' region
#pragma unroll
    for (int i = 0; i < NCR; ++i) {
      const int k = threadIdx.x + i * NT;
      if (k >= CA) continue;
      const int lx = k % CW, ly = k / CW, gx = x0 + lx, gy = y0 + ly;
      const int kb = (ly + 1) * BW + lx + 1;
      const bool in = inside(gx, gy);
#pragma unroll
      for (int part = 0; part < NP; ++part) {
        T d = (gx + 1 < nx ? qxs[part][kb] : T(0)) - (gx > 0 ? qxs[part][kb - 1] : T(0));
        d += (gy + 1 < ny ? qys[part][kb] : T(0)) - (gy > 0 ? qys[part][kb - BW] : T(0));
        if (tv3) d += (z + 1 < nz ? qzs[sl][part][kb] : T(0)) - (z > 0 ? qzs[sl ^ 1][part][kb] : T(0));
        ws[sl][part][k] = in ? fmaT(tau, d, vs[sl][part][(ly + 1) * AW + lx + 1]) : T(0);
      }
    }
    __syncthreads();
    // second step for the plane below, whose u' is complete now
    if (z > 0) step2_out(z - 1, tv3);
    // p'(z) on the tile for the next second step
    {
      const int kb = (ty + 1) * BW + tx + 1;
#pragma unroll
      for (int part = 0; part < NP; ++part) {
        pp1[0][part] = qxs[part][kb];
        pp1[1][part] = qys[part][kb];
        pp1[2][part] = qzs[sl][part][kb];
      }
    }
  }
  step2_out(nz - 1, false);
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

// K steps alternating between the dual sets a.p and a.q, then the final
// launch on the set the last step wrote.
template <class T, int NP>
hipError_t run_gp(GpArgs<T> a, int K, hipStream_t s, int* launches) {
  const dim3 g(ggrid((size_t)a.nx * a.ny * a.nz)), b(kGThreads);
  const dim3 gz((a.nx + kZX - 1) / kZX, (a.ny + zstep_rows<T>() - 1) / zstep_rows<T>()), bz(kZT);
  // FP32: pairs of steps in one launch, an odd step last on its own
  constexpr bool kPairs = sizeof(T) == 4;
  const dim3 gz2((a.nx + kZX - 1) / kZX, (a.ny + kZT / kZX - 1) / (kZT / kZX));
  (void)gz2;
  int nl = 0;
  for (int k = 0; k < K;) {
    a.first = k == 0 ? 1 : 0;
    int steps = 1;
    if constexpr (kPairs) {
      if (K - k >= 2) {
        hipLaunchKernelGGL((k_gp_zstep2<T, NP>), gz2, bz, 0, s, a);
        steps = 2;
      }
    }
    if (steps == 1) hipLaunchKernelGGL((k_gp_zstep<T, NP>), gz, bz, 0, s, a);
    k += steps;
    for (int d = 0; d < 3; ++d) std::swap(a.p[d], a.q[d]);
    ++nl;
  }
  a.first = K == 0 ? 1 : 0;
  hipLaunchKernelGGL((k_gp_final<T, NP>), g, b, 0, s, a);
  if (launches) *launches = nl + 1;
  return hipGetLastError();
}

}  // namespace

hipError_t launch_cprox(const ProxArgs& pa, hipStream_t s, int* launches) {
  GpArgs<float> a{};
  a.v = pa.v;
  a.x = pa.x;
  for (int k = 0; k < 3; ++k) a.vol[k] = pa.vol[k];
  a.st = pa.st;
  for (int k = 0; k < 3; ++k) {
    a.p[k] = pa.pa[k];
    a.q[k] = pa.pb[k];
  }
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
  for (int k = 0; k < 3; ++k) {
    a.p[k] = pa.p[k];
    a.q[k] = pa.p2[k];
  }
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
