// Fused-lasso proximal operator on gfx950: gradient projection on the dual of
// 3D isotropic TV denoising (Beck & Teboulle), then the soft threshold.
//
// With D the forward-difference operator along x, y, z (last difference on
// each axis zero) and u = v - tau D^T p, each dual step is
//     q = p + D u / (12 tau),   p = q / max(1, |q|)
// from p = 0; the result is soft(v - tau D^T p, step*l1).  -D^T p is the
// backward-difference divergence: div p(i) = sum_a p_a(i) - p_a(i - e_a), with
// p_a(i - e_a) = 0 on the first index and p_a = 0 on the last index of axis a.
//
// Temporal blocking.  A dual step at voxel i reads the previous dual at
// offsets in {-1, 0, 1} per axis, so L fused steps need an L-voxel halo.  A
// block owns a 64 x (W Q) tile in (x, y) -- one wavefront lane per x, Q = 4
// rows of y per lane, W = 12 wavefronts stacked in y -- and streams through z
// (one block per CU at up to 170 VGPRs).  The L steps
// form a pipeline along z: step l consumes the dual of step l-1 one plane
// behind it and keeps in registers, per point, the previous plane's dual and
// primal values.  Neighbours along x move with DPP wave shifts, along y through
// registers within a lane and through double-buffered LDS rows between
// wavefronts (one barrier per step and plane).  A kernel compiled for up to H
// fused steps has an H-voxel halo: points within H of the tile edge are
// computed but not stored, and tiles overlap by 2H.  The z-range is cut into
// chunks with an L+1 plane margin so that the grid fills the device.
//
// Boundaries: the z-component of the dual is exactly zero on the last plane
// (its z-difference is zero there, from p = 0 on) and the state below the first
// plane starts at zero, so the divergence carries no z masks; x / y masks are
// compiled only into the blocks whose tile touches the volume edge.
//
// One pass fuses up to H steps; a prox is a sequence of passes ping-ponging the
// dual between two buffers.  The last pass adds a half step (primal recovery),
// the soft threshold, the occupancy flags of the result and the store of x.
#include <algorithm>
#include <vector>

#include "rihvr_internal.h"

namespace rihvr {

constexpr int kTvWaves = 12;
constexpr int kTvQ = 4;                 // rows per lane
constexpr int kTvRX = 64;               // tile width (lanes)
constexpr int kTvRY = kTvWaves * kTvQ;  // tile height

struct TvPassArgs {
  const float* v;                 // nullptr: vol[st->prev]
  float* x;                       // nullptr: vol[st->next]
  float* vol[3];
  const float* pin[3];            // dual read by the first step (ignored when first)
  float* pout[3];                 // dual written by the last step (unless final)
  uint8_t* rowflag; uint8_t* planeflag;  // final pass: set where x != 0 (nullable)
  double* psum; double* ptv;      // final pass: per-block sum(x) and TV(x) of the stored x (nullable)
  const SolveState* st;
  int nx, ny, nz;
  int levels;                     // fused dual steps in this pass (<= H, <= H-1 when final)
  int first, final_, nonneg;
  int zchunk;                     // output planes per block
  float tau, c, thr;
  int gx, gy;                     // tiles along x and y (the grid of one frame)
};

// A register copy the compiler keeps (an identity DPP move).  The prefetched
// plane is copied out of its registers before they are reloaded; left to
// itself, the compiler renames the consumer onto the loaded registers, loads
// the next plane into fresh ones and moves them back at the loop's back edge,
// which waits for every load in flight.
__device__ __forceinline__ float vcopy(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xE4, 0xf, 0xf, false));
}
__device__ __forceinline__ float dpp_from_left(float v) {   // lane i <- lane i-1 (0 at lane 0)
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float dpp_from_right(float v) {  // lane i <- lane i+1 (0 at lane 63)
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xf, 0xf, true));
}

// Planes are addressed through buffer resources: a scalar descriptor of one
// plane (base, size in bytes) and a 32-bit per-lane byte offset.  A load at an
// offset past the plane returns 0 and a store there is dropped, so lanes
// outside the volume or outside the stored region use kTvOff.
constexpr unsigned kTvOff = 0x80000000u;
constexpr int kTvRsrcWord3 = 0x00020000;  // 32-bit data format, no stride / swizzle
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const float* base, size_t plane, size_t sz) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base) + plane * sz, (short)0, (int)(sz * 4),
                                           kTvRsrcWord3);
}
__device__ __forceinline__ float buf_ld(__amdgpu_buffer_rsrc_t r, unsigned off) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, unsigned off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, (int)off, 0, 0);
}

// Pass body.  H: the halo (tile geometry); LV: register slots for fused steps
// (H, or H - 1 on the final pass, which fuses at most H - 1).  EDGE: the tile
// touches the volume boundary, so every access and every difference is masked;
// interior tiles (most of them) skip the masks.  FIRST: the incoming dual is
// zero (nothing is read).  FINAL: the last pass (primal recovery and output)
// instead of storing the dual.
//
// With psum / ptv set, the final pass also sums x and its isotropic TV (forward
// differences, zero at the last index of each axis) over the points it stores.
// The differences of a plane need the next plane, so a plane's terms are taken
// when the next one is output (the last plane of the volume after the loop);
// the x+1 neighbour comes by a wave shift, the y+1 neighbour from the next row
// of the lane or, for the last row, from the next wave through LDS.  Every
// neighbour lies in the computed tile: the final pass fuses at most H - 1
// steps, so x is exact one point beyond the stored region.

template <int H, int LV, bool EDGE, bool FIRST, bool FINAL>
__device__ __forceinline__ void tv_pass_body(const TvPassArgs& A, int bx, int by, int bz,
                                             float (*s_py)[2][kTvWaves][64], float (*s_ut)[2][kTvWaves][64],
                                             float* s_v, float (*s_x)[kTvWaves][64], double (*s_red)[kTvWaves]) {
  constexpr int Q = kTvQ, NW = kTvWaves, NT = NW * 64;
  constexpr int IX = kTvRX - 2 * H, IY = kTvRY - 2 * H;  // interior (stored) extent
  const float* __restrict__ v = uniform_ptr(A.v ? A.v : pick3(A.vol[0], A.vol[1], A.vol[2], A.st->prev));
  float* __restrict__ xo = uniform_ptr(A.x ? A.x : pick3(A.vol[0], A.vol[1], A.vol[2], A.st->next));
  const int nx = A.nx, ny = A.ny, nz = A.nz;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int x = bx * IX - H + lane;
  const int ybase = by * IY - H + wv * Q;
  const bool inx = !EDGE || (x >= 0 && x < nx);
  const bool xlo = !EDGE || x > 0, xhi = !EDGE || x + 1 < nx;
  const bool ix_store = inx && lane >= H && lane < kTvRX - H;
  const size_t sz = (size_t)nx * ny;
  const int L = A.levels;
  const int zb = bz * A.zchunk, ze = min(nz, zb + A.zchunk);
  const int M = L + 1;
  const int zs = max(0, zb - M), zl = min(nz, ze + M);
  const float tau = A.tau, cc = A.c;

  bool ylo[Q], yhi[Q], ys[Q];
  unsigned off[Q];   // in-plane byte offset of the load (kTvOff outside the volume)
  unsigned offs[Q];  // ... of the store (kTvOff outside the stored interior)
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int y = ybase + q;
    const bool iny = !EDGE || (y >= 0 && y < ny);
    ylo[q] = !EDGE || y > 0;
    yhi[q] = !EDGE || y + 1 < ny;
    const int r = wv * Q + q;
    ys[q] = ix_store && iny && r >= H && r < kTvRY - H;
    off[q] = (inx && iny) ? (unsigned)(y * nx + x) * 4u : kTvOff;
    offs[q] = ys[q] ? off[q] : kTvOff;
  }
  // per fused step: previous plane's dual (3) and primal (1); final stage: previous p_z
  float Pp[LV][Q][3], Up[LV][Q], PzF[Q];
#pragma unroll
  for (int l = 0; l < LV; ++l)
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      Pp[l][q][0] = Pp[l][q][1] = Pp[l][q][2] = 0.f;
      Up[l][q] = 0.f;
    }
#pragma unroll
  for (int q = 0; q < Q; ++q) PzF[q] = 0.f;
  // objective pieces (final pass): x of the previous output plane, FP64 sums
  const bool obj = FINAL && A.psum != nullptr;
  float Xp[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) Xp[q] = 0.f;
  double s_acc = 0.0, t_acc = 0.0;
  // terms of the plane held in Xp; xn: the next plane (hz: it exists), slot:
  // the LDS slot holding the first row of every wave of the Xp plane
  auto accumulate = [&](const float (&xn)[Q], bool hz, int slot) {
    float ss = 0.f, tt = 0.f;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const float x0 = Xp[q];
      const float xr = dpp_from_right(x0);
      const float xu = (q < Q - 1) ? Xp[q + 1] : s_x[slot][wv < NW - 1 ? wv + 1 : wv][lane];
      const float gx = xhi ? xr - x0 : 0.f;
      const float gy = yhi[q] ? xu - x0 : 0.f;
      const float gz = hz ? xn[q] - x0 : 0.f;
      // per-voxel norm in FP32 (the hardware square root, within 1 ulp, not
      // the correctly rounded sequence), running sums in FP64
      const float t = __builtin_amdgcn_sqrtf(fmaf(gx, gx, fmaf(gy, gy, gz * gz)));
      ss += ys[q] ? fabsf(x0) : 0.f;   // ||x||_1
      tt += ys[q] ? t : 0.f;
    }
    s_acc += (double)ss;
    t_acc += (double)tt;
  };

  // Input planes are prefetched two ahead into two register sets used in
  // turn (the z loop is unrolled by two so that each set keeps its registers
  // and a set is read only after its loads, issued two planes earlier, are
  // done).  v of recent planes lives in a thread-private LDS ring
  // (slot = plane mod H+1).
  struct InPlane {
    float v[Q];
    float p[Q][3];
  };
  auto load_plane = [&](InPlane& P, int a) {
    const __amdgpu_buffer_rsrc_t rv = plane_rsrc(v, a, sz);
#pragma unroll
    for (int q = 0; q < Q; ++q) P.v[q] = buf_ld(rv, off[q]);
    if constexpr (!FIRST) {
      const __amdgpu_buffer_rsrc_t r0 = plane_rsrc(A.pin[0], a, sz);
      const __amdgpu_buffer_rsrc_t r1 = plane_rsrc(A.pin[1], a, sz);
      const __amdgpu_buffer_rsrc_t r2 = plane_rsrc(A.pin[2], a, sz);
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        P.p[q][0] = buf_ld(r0, off[q]);
        P.p[q][1] = buf_ld(r1, off[q]);
        P.p[q][2] = buf_ld(r2, off[q]);
      }
    }
  };
  auto vring = [&](int a, int q) -> float& { return s_v[((a % (H + 1)) * Q + q) * NT + threadIdx.x]; };

  // Arrival of the previous dual c3 at plane a for fused step l: u(a), then
  // the dual step at plane a - 1 (which needs u(a) for its z-difference).
  auto arrive = [&](int l, int a, int par, float (&c3)[Q][3]) {
    float un[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) un[q] = vring(a, q);  // thread-private: read before the barrier
    s_py[l][par][wv][lane] = c3[Q - 1][1];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const float pxm = dpp_from_left(c3[q][0]);
      const float pym = (q > 0) ? c3[q - 1][1] : s_py[l][par][wv > 0 ? wv - 1 : 0][lane];
      float d = (xhi ? c3[q][0] : 0.f) - (xlo ? pxm : 0.f);
      d += (yhi[q] ? c3[q][1] : 0.f) - (ylo[q] ? pym : 0.f);
      d += c3[q][2] - Pp[l][q][2];
      un[q] = fmaf(tau, d, un[q]);
    }
    if (a > zs) {
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const float u0 = Up[l][q];
        const float uxp = dpp_from_right(u0);
        const float uyp = (q < Q - 1) ? Up[l][q + 1] : s_ut[l][par ^ 1][wv < NW - 1 ? wv + 1 : wv][lane];
        const float gx = xhi ? uxp - u0 : 0.f;
        const float gy = yhi[q] ? uyp - u0 : 0.f;
        const float gz = un[q] - u0;       // plane a exists
        const float qx = fmaf(cc, gx, Pp[l][q][0]);
        const float qy = fmaf(cc, gy, Pp[l][q][1]);
        const float qz = fmaf(cc, gz, Pp[l][q][2]);
        const float n2 = fmaf(qx, qx, fmaf(qy, qy, qz * qz));
        const float sc = fminf(1.f, __frsqrt_rn(n2));   // 1 / max(1, |q|)
        Pp[l][q][0] = c3[q][0];
        Pp[l][q][1] = c3[q][1];
        Pp[l][q][2] = c3[q][2];
        c3[q][0] = qx * sc;
        c3[q][1] = qy * sc;
        c3[q][2] = qz * sc;
      }
      // Up is read by the neighbours above (q+1) before it is replaced
#pragma unroll
      for (int q = 0; q < Q; ++q) Up[l][q] = un[q];
    } else {
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        Pp[l][q][0] = c3[q][0];
        Pp[l][q][1] = c3[q][1];
        Pp[l][q][2] = c3[q][2];
        Up[l][q] = un[q];
      }
    }
    s_ut[l][par][wv][lane] = un[0];
  };
  // Flush of fused step l: dual step at the last plane zl - 1 (no plane above).
  auto flush = [&](int l, int par, float (&c3)[Q][3]) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const float u0 = Up[l][q];
      const float uxp = dpp_from_right(u0);
      const float uyp = (q < Q - 1) ? Up[l][q + 1] : s_ut[l][par ^ 1][wv < NW - 1 ? wv + 1 : wv][lane];
      const float gx = xhi ? uxp - u0 : 0.f;
      const float gy = yhi[q] ? uyp - u0 : 0.f;
      const float qx = fmaf(cc, gx, Pp[l][q][0]);
      const float qy = fmaf(cc, gy, Pp[l][q][1]);
      const float qz = Pp[l][q][2];
      const float n2 = fmaf(qx, qx, fmaf(qy, qy, qz * qz));
      const float sc = fminf(1.f, __frsqrt_rn(n2));
      c3[q][0] = qx * sc;
      c3[q][1] = qy * sc;
      c3[q][2] = qz * sc;
    }
  };
  // Output stage: the dual of the last fused step at plane m (stored), or on
  // the final pass the primal recovery, soft threshold, store and flags.
  auto output = [&](int m, int par, float (&c3)[Q][3]) {
    const bool zstore = m >= zb && m < ze;
    if constexpr (!FINAL) {
      if (zstore) {
        const __amdgpu_buffer_rsrc_t o0 = plane_rsrc(A.pout[0], m, sz);
        const __amdgpu_buffer_rsrc_t o1 = plane_rsrc(A.pout[1], m, sz);
        const __amdgpu_buffer_rsrc_t o2 = plane_rsrc(A.pout[2], m, sz);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          buf_st(o0, offs[q], c3[q][0]);
          buf_st(o1, offs[q], c3[q][1]);
          buf_st(o2, offs[q], c3[q][2]);
        }
      }
    } else {
      float vm[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) vm[q] = vring(m, q);  // thread-private: read before the barrier
      s_py[H][par][wv][lane] = c3[Q - 1][1];
      __syncthreads();
      const __amdgpu_buffer_rsrc_t rx = plane_rsrc(xo, m, sz);
      float xs[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        float u = vm[q];
        if (tau != 0.f) {
          const float pxm = dpp_from_left(c3[q][0]);
          const float pym = (q > 0) ? c3[q - 1][1] : s_py[H][par][wv > 0 ? wv - 1 : 0][lane];
          float d = (xhi ? c3[q][0] : 0.f) - (xlo ? pxm : 0.f);
          d += (yhi[q] ? c3[q][1] : 0.f) - (ylo[q] ? pym : 0.f);
          d += c3[q][2] - PzF[q];
          u = fmaf(tau, d, u);
        }
        PzF[q] = c3[q][2];
        float xv;
        if (A.nonneg) {
          xv = fmaxf(u - A.thr, 0.f);
        } else {
          xv = copysignf(fmaxf(fabsf(u) - A.thr, 0.f), u);
        }
        xs[q] = xv;
        const bool st = zstore && ys[q];
        if (zstore) buf_st(rx, offs[q], xv);
        if (A.rowflag != nullptr) {
          const bool nzr = __ballot(st && xv != 0.f) != 0;
          if (nzr && lane == 0) {
            A.rowflag[(size_t)m * ny + ybase + q] = 1;
            A.planeflag[m] = 1;
          }
        }
      }
      if (obj) {
        // plane m - 1 is complete now; its first rows went to slot par ^ 1
        if (m - 1 >= zb && m - 1 < ze) accumulate(xs, true, par ^ 1);
        s_x[par][wv][lane] = xs[0];  // read after the next output's barrier
#pragma unroll
        for (int q = 0; q < Q; ++q) Xp[q] = xs[q];
      }
    }
  };

  // Steady part: plane a1 = zs + s arrives (a1 < zl), every fused step is an
  // arrival or idle; the planes two ahead are being loaded meanwhile.
  auto step = [&](int s, InPlane& P) {
    const int par = s & 1;
    const int a1 = zs + s;
    float c3[Q][3];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      vring(a1, q) = vcopy(P.v[q]);
      c3[q][0] = FIRST ? 0.f : vcopy(P.p[q][0]);
      c3[q][1] = FIRST ? 0.f : vcopy(P.p[q][1]);
      c3[q][2] = FIRST ? 0.f : vcopy(P.p[q][2]);
    }
    if (a1 + 2 < zl) load_plane(P, a1 + 2);
#pragma unroll
    for (int l = 0; l < LV; ++l) {
      if (l >= L) break;
      const int a = a1 - l;
      if (a < zs) break;                  // this and the later steps are idle
      arrive(l, a, par, c3);
    }
    const int m = a1 - L;
    if (m >= zs) output(m, par, c3);
  };

  InPlane PA, PB;
  load_plane(PA, zs);
  if (zs + 1 < zl) load_plane(PB, zs + 1);
  const int s_main = zl - zs;
  for (int s = 0; s < s_main; s += 2) {
    step(s, PA);
    if (s + 1 < s_main) step(s + 1, PB);
  }
  // Drain: no plane arrives; fused step l flushes at s = s_main + l.
  const int nsteps = s_main + L;
  for (int s = s_main; s < nsteps; ++s) {
    const int par = s & 1;
    const int a1 = zs + s;
    float c3[Q][3];
#pragma unroll
    for (int q = 0; q < Q; ++q) c3[q][0] = c3[q][1] = c3[q][2] = 0.f;
#pragma unroll
    for (int l = 0; l < LV; ++l) {
      if (l >= L) break;
      const int a = a1 - l;
      if (a > zl) continue;               // already flushed
      if (a < zs) break;
      if (a == zl) flush(l, par, c3);
      else arrive(l, a, par, c3);
    }
    const int m = a1 - L;
    if (m >= zs && m < zl) output(m, par, c3);
  }
  if constexpr (FINAL) {
    if (obj) {
      if (ze == nz) {
        // the last plane of the volume: no plane above it (its z-difference is 0)
        __syncthreads();
        accumulate(Xp, false, (nsteps - 1) & 1);
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        s_acc += __shfl_xor(s_acc, off, 64);
        t_acc += __shfl_xor(t_acc, off, 64);
      }
      if (lane == 0) {
        s_red[0][wv] = s_acc;
        s_red[1][wv] = t_acc;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        double s = 0.0, t = 0.0;
        for (int w = 0; w < NW; ++w) {
          s += s_red[0][w];
          t += s_red[1][w];
        }
        const size_t blk = (size_t)bx + (size_t)A.gx * ((size_t)by + (size_t)A.gy * bz);
        A.psum[blk] = s;
        A.ptv[blk] = t;
      }
    }
  }
}

template <int H>
__device__ __forceinline__ void tv_pass_entry(const TvPassArgs& A, int bx, int by, int bz) {
  __shared__ float s_py[H + 1][2][kTvWaves][64];  // bottom-row p_y per wave, per step, parity
  __shared__ float s_ut[H][2][kTvWaves][64];      // top-row u per wave, per step, parity
  __shared__ float s_v[(H + 1) * kTvQ * kTvWaves * 64];  // v ring, thread-private
  __shared__ float s_x[2][kTvWaves][64];          // final pass: first-row x per wave, parity
  __shared__ double s_red[2][kTvWaves];           // final pass: per-wave sums
  if (A.st != nullptr && A.st->done) return;
  constexpr int IX = kTvRX - 2 * H, IY = kTvRY - 2 * H;
  const int x0 = bx * IX - H, y0 = by * IY - H;
  // interior tile: every point of the region and its +-1 neighbours lie inside
  const bool interior = x0 >= 1 && x0 + kTvRX <= A.nx - 1 && y0 >= 1 && y0 + kTvRY <= A.ny - 1;
#define RIHVR_TV_BODY(E, F, FIN) \
  tv_pass_body<H, (FIN) ? H - 1 : H, E, F, FIN>(A, bx, by, bz, s_py, s_ut, s_v, s_x, s_red)
  if (A.final_) {
    if (A.first) {
      if (interior) RIHVR_TV_BODY(false, true, true);
      else RIHVR_TV_BODY(true, true, true);
    } else {
      if (interior) RIHVR_TV_BODY(false, false, true);
      else RIHVR_TV_BODY(true, false, true);
    }
  } else {
    if (A.first) {
      if (interior) RIHVR_TV_BODY(false, true, false);
      else RIHVR_TV_BODY(true, true, false);
    } else {
      if (interior) RIHVR_TV_BODY(false, false, false);
      else RIHVR_TV_BODY(true, false, false);
    }
  }
#undef RIHVR_TV_BODY
}

// The second launch-bounds argument is the minimum number of waves per SIMD
// the register allocation must allow: 12-wave blocks need 3 (<= 170 VGPRs,
// one block per CU), which every fusion depth fits.
constexpr int kTvWavesPerSimd = (kTvWaves + 3) / 4;

template <int H>
__global__ void __launch_bounds__(kTvWaves * 64, kTvWavesPerSimd) k_tv_pass(TvPassArgs A) {
  const uint32_t n = gridDim.x * gridDim.y * gridDim.z;
  const uint32_t t = xcd_tile(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z), n);
  tv_pass_entry<H>(A, t % A.gx, (t / A.gx) % A.gy, t / (A.gx * A.gy));
}

template <int H>
__global__ void __launch_bounds__(kTvWaves * 64, kTvWavesPerSimd) k_tv_pass_b(const TvPassArgs* __restrict__ args,
                                                                                  BatchMap map) {
  const uint32_t b = xcd_tile(blockIdx.x, gridDim.x);
  int lo = 0, hi = map.n;  // largest f with offs[f] <= b
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (map.offs[mid] <= b) lo = mid;
    else hi = mid;
  }
  lo = __builtin_amdgcn_readfirstlane(lo);  // uniform: the frame's arguments come in as scalar loads
  const TvPassArgs A = args[lo];
  const int lb = (int)(b - (uint32_t)__builtin_amdgcn_readfirstlane(map.offs[lo]));
  tv_pass_entry<H>(A, lb % A.gx, (lb / A.gx) % A.gy, lb / (A.gx * A.gy));
}

// Blocks of one pass: x tiles, y tiles, z chunks.  The z-range is cut into
// chunks of at least 16 planes until the grid holds about `want` blocks.
static void pass_grid(int nx, int ny, int nz, int H, int want, dim3* grid, int* zchunk) {
  const int tx = (nx + (kTvRX - 2 * H) - 1) / (kTvRX - 2 * H);
  const int ty = (ny + (kTvRY - 2 * H) - 1) / (kTvRY - 2 * H);
  const int nzc = std::max(1, std::min(nz / 16, (want + tx * ty - 1) / (tx * ty)));
  const int zc = (nz + nzc - 1) / nzc;
  *zchunk = zc;
  *grid = dim3(tx, ty, (nz + zc - 1) / zc);
}

static int clamp_levels(int H) { return H < kTvLevelsMin ? kTvDefaultLevels : std::min(H, kTvLevelsMax); }

int prox_passes(int inner_iters, double tau, int levels) {
  if (!(tau > 0.0) || inner_iters <= 0) return 1;
  const int H = clamp_levels(levels);
  return (inner_iters + 1 + H - 1) / H;   // K dual steps + one primal half step
}

size_t tv_pass_args_size() { return sizeof(TvPassArgs); }

int tv_pass_blocks(int nx, int ny, int nz, int levels, int blocks) {
  dim3 g;
  int zc = 0;
  pass_grid(nx, ny, nz, clamp_levels(levels), blocks > 0 ? blocks : kTvDefaultBlocks, &g, &zc);
  return (int)(g.x * g.y * g.z);
}

int tv_blocks_bound(int nx, int ny, int nz) {
  // the most tiles (deepest halo) times the most z chunks pass_grid makes
  const int tx = (nx + (kTvRX - 2 * kTvLevelsMax) - 1) / (kTvRX - 2 * kTvLevelsMax);
  const int ty = (ny + (kTvRY - 2 * kTvLevelsMax) - 1) / (kTvRY - 2 * kTvLevelsMax);
  return tx * ty * std::max(1, nz / 16);
}

int tv_pass_zchunk(int nx, int ny, int nz, int levels, int blocks) {
  dim3 g;
  int zc = 0;
  pass_grid(nx, ny, nz, clamp_levels(levels), blocks > 0 ? blocks : kTvDefaultBlocks, &g, &zc);
  return zc;
}

// Argument structs of every pass of one prox application.  Dual steps per
// pass: non-final passes take H, the final pass the rest (at most H - 1,
// leaving room for the primal half step in its halo).
int prox_pass_args(const ProxArgs& pa, void* out, int* blocks_per_pass) {
  const double tau = pa.step * pa.tv;
  const double thr = pa.step * pa.l1;
  const bool use_tv = tau > 0.0 && pa.inner_iters > 0;
  const int K = use_tv ? pa.inner_iters : 0;
  const int H = clamp_levels(pa.levels);
  const int npass = prox_passes(K, tau, H);
  TvPassArgs a{};
  a.v = pa.v;
  a.x = pa.x;
  for (int k = 0; k < 3; ++k) a.vol[k] = pa.vol[k];
  a.rowflag = pa.rowflag;
  a.planeflag = pa.planeflag;
  a.psum = pa.psum;
  a.ptv = pa.ptv;
  a.st = pa.st;
  a.nx = pa.nx; a.ny = pa.ny; a.nz = pa.nz;
  a.nonneg = pa.nonneg;
  a.tau = (float)tau;
  a.c = use_tv ? (float)(1.0 / (12.0 * tau)) : 0.f;
  a.thr = (float)thr;
  dim3 grid;
  pass_grid(pa.nx, pa.ny, pa.nz, H, pa.blocks > 0 ? pa.blocks : kTvDefaultBlocks, &grid, &a.zchunk);
  a.gx = grid.x;
  a.gy = grid.y;
  if (blocks_per_pass) *blocks_per_pass = grid.x * grid.y * grid.z;
  TvPassArgs* o = static_cast<TvPassArgs*>(out);
  int done = 0;
  for (int p = 0; p < npass; ++p) {
    const bool fin = p == npass - 1;
    const int lv = fin ? K - done : std::min(H, K - done);
    a.levels = lv;
    a.first = (done == 0) ? 1 : 0;
    a.final_ = fin ? 1 : 0;
    float* const* src = (p & 1) ? pa.pb : pa.pa;
    float* const* dst = (p & 1) ? pa.pa : pa.pb;
    for (int k = 0; k < 3; ++k) {
      a.pin[k] = src[k];
      a.pout[k] = dst[k];
    }
    o[p] = a;
    done += lv;
  }
  return npass;
}

hipError_t launch_prox(const ProxArgs& pa, hipStream_t s, int* launches) {
  const double tau = pa.step * pa.tv;
  const int K = (tau > 0.0 && pa.inner_iters > 0) ? pa.inner_iters : 0;
  const int H = clamp_levels(pa.levels);
  std::vector<TvPassArgs> args(prox_passes(K, tau, H));
  int nb = 0;
  const int npass = prox_pass_args(pa, args.data(), &nb);
  const dim3 grid(args[0].gx, args[0].gy, (nb / (args[0].gx * args[0].gy)));
  for (int p = 0; p < npass; ++p) {
    switch (H) {
      case 2: hipLaunchKernelGGL(k_tv_pass<2>, grid, dim3(kTvWaves * 64), 0, s, args[p]); break;
      case 3: hipLaunchKernelGGL(k_tv_pass<3>, grid, dim3(kTvWaves * 64), 0, s, args[p]); break;
      default: hipLaunchKernelGGL(k_tv_pass<4>, grid, dim3(kTvWaves * 64), 0, s, args[p]); break;
    }
  }
  if (launches) *launches = npass;
  return hipGetLastError();
}

hipError_t launch_tv_pass_batched(int levels, const void* args, BatchMap map, int nblocks, hipStream_t s) {
  const TvPassArgs* a = static_cast<const TvPassArgs*>(args);
  switch (clamp_levels(levels)) {
    case 2: hipLaunchKernelGGL(k_tv_pass_b<2>, dim3(nblocks), dim3(kTvWaves * 64), 0, s, a, map); break;
    case 3: hipLaunchKernelGGL(k_tv_pass_b<3>, dim3(nblocks), dim3(kTvWaves * 64), 0, s, a, map); break;
    default: hipLaunchKernelGGL(k_tv_pass_b<4>, dim3(nblocks), dim3(kTvWaves * 64), 0, s, a, map); break;
  }
  return hipGetLastError();
}

}  // namespace rihvr
