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
// Per-plane 2D TV (TV2): the TV of the paper's Eq. (4) taken in every plane on
// its own.  The dual has no z component (neither read nor stored), the step is
// 1/(8 tau) and planes do not couple, so chunks need no z margin.
//
// Dual storage in bfloat16 (dual_bf16): the dual between passes is rounded to
// bfloat16 (to nearest, ties to even) when stored and widened when read; the
// arithmetic stays FP32.  The dual lies in the unit ball, so its bytes halve
// at 2^-9 relative precision.
//
// FGP (accelerated dual iteration): every dual pass takes one step at the
// extrapolated point r, reads (r, p_prev) and stores (p, r_next), r_next =
// p + w (p - p_prev) with w = (t_k - 1)/t_{k+1} of the FISTA sequence (set per
// pass by the host); the final pass steps at r like a plain pass.
//
// Boundaries: the z-component of the dual is exactly zero on the last plane
// (its z-difference is zero there, from p = 0 on) and the state below the first
// plane starts at zero, so the divergence carries no z masks; x / y masks are
// compiled only into the blocks whose tile touches the volume edge.
//
// One pass fuses up to H steps; a prox is a sequence of passes ping-ponging the
// dual between two buffers.  The last pass adds a half step (primal recovery),
// the soft threshold, the occupancy flags of the result and the store of x.
// It runs its own kernel whose tile has an (H+1)-voxel halo: x at a voxel needs
// the dual one voxel below it on every axis, and the objective's differences
// need x one voxel above, so with one more voxel of halo the last pass fuses
// a full H dual steps as well (K steps take ceil(K/H) passes).
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
  int levels;                     // fused dual steps in this pass (<= H)
  int first, final_, nonneg;
  int tv2;                        // per-plane 2D TV (no z component, no z margin)
  int keep_dual;                  // final pass: also store the dual to pout (warm start of the next prox)
  int flip_npass;                 // > 0: the solve's passes ping-pong the dual across outer iterations;
                                  // pin and pout trade places when (st->it - 1) * flip_npass is odd
  int dual_bf16;                  // the dual buffers hold bfloat16
  const float* pin2[3];           // FGP: p_prev read with r (= pin)
  float* pout2[3];                // FGP: p written beside r_next (= pout)
  float fgp_w;                    // FGP: extrapolation weight of this pass
  RowStores rs;                   // final pass with rs.on: x_{k+1} into row store st->scur ^ 1
  int fgp;                        // FGP dual pass (one step; never the final pass)
  int zchunk;                     // output planes per block (the first nfull tiles)
  int nfull;                      // tiles (in raster order) cut into chunks of zchunk planes; the
  int zchunk2;                    // remaining gx*gy - nfull tiles are cut into chunks of zchunk2
  int nblocks;                    // blocks of the pass (the objective partials are per block)
  float tau, c, thr;
  int gx, gy;                     // tiles along x and y (the grid of one frame)
  size_t zoff_v, zoff_x;          // grouped per-plane prox: first plane of the group in v and x (elements)
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

// Dual planes, FP32 or bfloat16 (`bf`, uniform).  Offsets are those of the
// FP32 layout; a bfloat16 element sits at half of it (kTvOff / 2 is still past
// every plane).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t dual_rsrc(const float* base, size_t plane, size_t sz, bool bf) {
  if (!bf) return plane_rsrc(base, plane, sz);
  const uint16_t* b = reinterpret_cast<const uint16_t*>(base) + plane * sz;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint16_t*>(b), (short)0, (int)(sz * 2), kTvRsrcWord3);
}
__device__ __forceinline__ float dual_ld(__amdgpu_buffer_rsrc_t r, unsigned off, bool bf) {
  if (!bf) return buf_ld(r, off);
  const unsigned short h = __builtin_amdgcn_raw_buffer_load_b16(r, (int)(off >> 1), 0, 0);
  return __uint_as_float((unsigned)h << 16);
}
__device__ __forceinline__ void dual_st(__amdgpu_buffer_rsrc_t r, unsigned off, float v, bool bf) {
  if (!bf) {
    buf_st(r, off, v);
    return;
  }
  const unsigned u = __float_as_uint(v);
  const unsigned h = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;   // round to nearest, ties to even (|v| <= 1)
  __builtin_amdgcn_raw_buffer_store_b16((unsigned short)h, r, (int)(off >> 1), 0, 0);
}

// Pass body.  H: the halo (tile geometry); LV: register slots for fused steps
// (the halo on dual passes; on the final pass, whose halo is one wider, H - 1).  EDGE: the tile
// touches the volume boundary, so every access and every difference is masked;
// interior tiles (most of them) skip the masks.  TV2: per-plane 2D TV.  FIRST: the incoming dual is
// zero (nothing is read).  FINAL: the last pass (primal recovery and output)
// instead of storing the dual.  FGP: a one-step accelerated dual pass (above).
//
// With psum / ptv set, the final pass also sums x and its isotropic TV (forward
// differences, zero at the last index of each axis) over the points it stores.
// The differences of a plane need the next plane, so a plane's terms are taken
// when the next one is output (the last plane of the volume after the loop);
// the x+1 neighbour comes by a wave shift, the y+1 neighbour from the next row
// of the lane or, for the last row, from the next wave through LDS.  Every
// neighbour lies in the computed tile: the final pass fuses at most H - 1
// steps for its halo of H, so x is exact one point beyond the stored region.

// Bound on a wave's wait for another segment to publish a row-store index
// (about 2^20 * 128 clocks; the publisher needs a few hundred).
constexpr int kStoreSpinLimit = 1 << 20;

template <int H, int LV, bool EDGE, bool FIRST, bool FINAL, bool TV2, bool FGP, bool BF, bool SP>
__device__ __forceinline__ void tv_pass_body(const TvPassArgs& A, int bx, int by, int zb, int ze, int blk,
                                             float (*s_py)[2][kTvWaves][64], float (*s_ut)[2][kTvWaves][64],
                                             float* s_v, float (*s_x)[kTvWaves][64], double (*s_red)[kTvWaves],
                                             float* s_fin, double* s_sum) {
  constexpr int Q = kTvQ, NW = kTvWaves, NT = NW * 64;
  constexpr int IX = kTvRX - 2 * H, IY = kTvRY - 2 * H;  // interior (stored) extent
  const float* __restrict__ v =
      uniform_ptr((A.v ? A.v : pick3(A.vol[0], A.vol[1], A.vol[2], A.st->prev)) + A.zoff_v);
  float* __restrict__ xo = uniform_ptr((A.x ? A.x : pick3(A.vol[0], A.vol[1], A.vol[2], A.st->next)) + A.zoff_x);
  const int nx = A.nx, ny = A.ny, nz = A.nz;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // dual buffers of this pass: with a warm-started dual the sets alternate
  // from one outer iteration to the next when a prox has an odd number of passes
  const bool flip = A.flip_npass > 0 && A.st != nullptr && (((A.st->it - 1) * A.flip_npass) & 1);
  const float* pin[3];
  float* pout[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    pin[k] = uniform_ptr(flip ? const_cast<const float*>(A.pout[k]) : A.pin[k]);
    pout[k] = uniform_ptr(flip ? const_cast<float*>(A.pin[k]) : A.pout[k]);
  }
  constexpr bool bf = BF;   // dual buffers in bfloat16
  const int x = bx * IX - H + lane;
  const int ybase = by * IY - H + wv * Q;
  const bool inx = !EDGE || (x >= 0 && x < nx);
  const bool xlo = !EDGE || x > 0, xhi = !EDGE || x + 1 < nx;
  const bool ix_store = inx && lane >= H && lane < kTvRX - H;
  const size_t sz = (size_t)nx * ny;
  const int L = A.levels;

  const int M = TV2 ? 0 : L + 1;
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
  // per fused step: previous plane's dual (3) and primal (1)
  float Pp[LV][Q][3], Up[LV][Q];
#pragma unroll
  for (int l = 0; l < LV; ++l)
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      Pp[l][q][0] = Pp[l][q][1] = Pp[l][q][2] = 0.f;
      Up[l][q] = 0.f;
    }
  // Final-pass state kept in thread-private LDS rather than registers (the
  // final pass holds H fused steps in a tile of halo H + 1 and would spill):
  // the previous output plane's p_z (PzF) and x (Xp), and the FP64 sums of
  // ||x||_1 and TV(x) (objective pieces).
  auto PzF = [&](int q) -> float& { return s_fin[q * NT + threadIdx.x]; };
  auto Xp = [&](int q) -> float& { return s_fin[(Q + q) * NT + threadIdx.x]; };
  const bool obj = FINAL && A.psum != nullptr;
  if constexpr (FINAL) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      PzF(q) = 0.f;
      Xp(q) = 0.f;
    }
    s_sum[threadIdx.x] = 0.0;
    s_sum[NT + threadIdx.x] = 0.0;
  }
  // terms of the plane held in Xp; xn: the next plane (hz: it exists), slot:
  // the LDS slot holding the first row of every wave of the Xp plane
  auto accumulate = [&](const float* xn, bool hz, int slot) {
    float ss = 0.f, tt = 0.f;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const float x0 = Xp(q);
      const float xr = dpp_from_right(x0);
      const float xu = (q < Q - 1) ? Xp(q + 1) : s_x[slot][wv < NW - 1 ? wv + 1 : wv][lane];
      const float gx = xhi ? xr - x0 : 0.f;
      const float gy = yhi[q] ? xu - x0 : 0.f;
      const float gz = (hz && !TV2) ? xn[q] - x0 : 0.f;
      // per-voxel norm in FP32 (the hardware square root, within 1 ulp, not
      // the correctly rounded sequence), running sums in FP64
      const float t = __builtin_amdgcn_sqrtf(fmaf(gx, gx, fmaf(gy, gy, gz * gz)));
      ss += ys[q] ? fabsf(x0) : 0.f;   // ||x||_1
      tt += ys[q] ? t : 0.f;
    }
    s_sum[threadIdx.x] += (double)ss;
    s_sum[NT + threadIdx.x] += (double)tt;
  };

  // Input planes are prefetched two ahead into two register sets used in
  // turn (the z loop is unrolled by two so that each set keeps its registers
  // and a set is read only after its loads, issued two planes earlier, are
  // done).  v of recent planes lives in a thread-private LDS ring
  // (slot = plane mod H+1).
  struct InPlane {
    float v[Q];
    float p[Q][3];
    float pp[Q][3];   // FGP: p_prev of the plane
  };
  auto load_plane = [&](InPlane& P, int a) {
    const __amdgpu_buffer_rsrc_t rv = plane_rsrc(v, a, sz);
#pragma unroll
    for (int q = 0; q < Q; ++q) P.v[q] = buf_ld(rv, off[q]);
    if constexpr (!FIRST) {
      const __amdgpu_buffer_rsrc_t r0 = dual_rsrc(pin[0], a, sz, bf);
      const __amdgpu_buffer_rsrc_t r1 = dual_rsrc(pin[1], a, sz, bf);
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        P.p[q][0] = dual_ld(r0, off[q], bf);
        P.p[q][1] = dual_ld(r1, off[q], bf);
      }
      if constexpr (!TV2) {
        const __amdgpu_buffer_rsrc_t r2 = dual_rsrc(pin[2], a, sz, bf);
#pragma unroll
        for (int q = 0; q < Q; ++q) P.p[q][2] = dual_ld(r2, off[q], bf);
      } else {
#pragma unroll
        for (int q = 0; q < Q; ++q) P.p[q][2] = 0.f;
      }
      if constexpr (FGP) {
        const __amdgpu_buffer_rsrc_t s0 = dual_rsrc(A.pin2[0], a, sz, bf);
        const __amdgpu_buffer_rsrc_t s1 = dual_rsrc(A.pin2[1], a, sz, bf);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          P.pp[q][0] = dual_ld(s0, off[q], bf);
          P.pp[q][1] = dual_ld(s1, off[q], bf);
          P.pp[q][2] = 0.f;
        }
        if constexpr (!TV2) {
          const __amdgpu_buffer_rsrc_t s2 = dual_rsrc(A.pin2[2], a, sz, bf);
#pragma unroll
          for (int q = 0; q < Q; ++q) P.pp[q][2] = dual_ld(s2, off[q], bf);
        }
      }
    }
  };
  auto vring = [&](int a, int q) -> float& { return s_v[((a % (LV + 1)) * Q + q) * NT + threadIdx.x]; };

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
      if constexpr (!TV2) d += c3[q][2] - Pp[l][q][2];
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
        const float qz = TV2 ? 0.f : fmaf(cc, gz, Pp[l][q][2]);
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
      const float qz = TV2 ? 0.f : Pp[l][q][2];
      const float n2 = fmaf(qx, qx, fmaf(qy, qy, qz * qz));
      const float sc = fminf(1.f, __frsqrt_rn(n2));
      c3[q][0] = qx * sc;
      c3[q][1] = qy * sc;
      c3[q][2] = qz * sc;
    }
  };
  // Output stage: the dual of the last fused step at plane m (stored), or on
  // the final pass the primal recovery, soft threshold, store and flags.
  auto store3 = [&](float* const* dst, int m, const float (&c3)[Q][3]) {
    const __amdgpu_buffer_rsrc_t o0 = dual_rsrc(dst[0], m, sz, bf);
    const __amdgpu_buffer_rsrc_t o1 = dual_rsrc(dst[1], m, sz, bf);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      dual_st(o0, offs[q], c3[q][0], bf);
      dual_st(o1, offs[q], c3[q][1], bf);
    }
    if constexpr (!TV2) {
      const __amdgpu_buffer_rsrc_t o2 = dual_rsrc(dst[2], m, sz, bf);
#pragma unroll
      for (int q = 0; q < Q; ++q) dual_st(o2, offs[q], c3[q][2], bf);
    }
  };
  // FGP: p_prev of the plane that arrived last (the next plane to be output)
  float PPv[Q][3];
#pragma unroll
  for (int q = 0; q < Q; ++q) PPv[q][0] = PPv[q][1] = PPv[q][2] = 0.f;
  auto store_dual = [&](int m, const float (&c3)[Q][3]) {
    if constexpr (FGP) {
      // c3 is p at plane m; the next pass steps at r_next = p + w (p - p_prev)
      const float w = A.fgp_w;
      float rn[Q][3];
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int k = 0; k < 3; ++k) rn[q][k] = fmaf(w, c3[q][k] - PPv[q][k], c3[q][k]);
      store3(pout, m, rn);
      store3(A.pout2, m, c3);
    } else {
      store3(pout, m, c3);
    }
  };
  // Row-compressed store of x_{k+1} (A.rs.on): this wave's segments of rows
  // ybase .. ybase + Q - 1 of plane m; bit q of nzm: segment q holds a
  // non-zero value.  Lane q claims row q's slot (-1 -> -2) when it is still
  // absent; the claimed rows take consecutive pool rows with one counter
  // update and their indices are published; a row found claimed by another
  // segment is waited for (its claimer depends on nothing, so the wait ends;
  // a bound on it reports an overflow instead).  Slot -3: the pool ran out.
  // Pool rows not in use are zero (zeroed at the start and when a store is
  // recycled), so a segment writes only its values and no ordering beyond the
  // slots' atomics is needed; every occupied row takes exactly one pool row.
  auto store_rows = [&](int m, const float (&xs)[Q], unsigned nzm, bool zstore) {
    const int k = A.st->scur ^ 1;
    float* pool = k == 0 ? A.rs.pool[0] : A.rs.pool[1];
    const bool mine = lane < Q && ((nzm >> lane) & 1u);
    int32_t* tab = (k == 0 ? A.rs.slot[0] : A.rs.slot[1]) + (size_t)m * ny + (mine ? ybase + lane : 0);
    int idx = -1;
    if (mine) idx = __hip_atomic_load(tab, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (mine && idx == -1) {
      idx = atomicCAS(tab, -1, -2);
      idx = idx == -1 ? -4 : idx;          // -4: this lane won the claim
    }
    const uint64_t wm = __ballot(mine && idx == -4);
    if (wm != 0) {
      uint32_t base = 0;
      if (lane == 0) base = atomicAdd(&A.rs.count[k], (uint32_t)__popcll(wm));
      base = __builtin_amdgcn_readfirstlane(base);
      if (mine && idx == -4) {
        const uint32_t sn = base + (uint32_t)__popcll(wm & ((1ull << lane) - 1ull));
        idx = sn < A.rs.cap ? (int)sn : -3;
        if (idx < 0) atomicOr(A.rs.overflow, 1u);
        __hip_atomic_store(tab, idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    for (int spin = 0; __ballot(mine && idx == -2) != 0; ++spin) {
      if (spin >= kStoreSpinLimit) {
        if (mine && idx == -2) {
          atomicOr(A.rs.overflow, 2u);
          idx = -3;
        }
        break;
      }
      __builtin_amdgcn_s_sleep(2);
      if (mine && idx == -2) idx = __hip_atomic_load(tab, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      if (!((nzm >> q) & 1u)) continue;
      const int r = __builtin_amdgcn_readlane(idx, q);
      if (r >= 0 && zstore && ys[q]) pool[(size_t)r * nx + x] = xs[q];
    }
  };
  auto output = [&](int m, int par, float (&c3)[Q][3]) {
    const bool zstore = m >= zb && m < ze;
    if constexpr (!FINAL) {
      if (zstore) store_dual(m, c3);
    } else {
      if (A.keep_dual && zstore) store_dual(m, c3);
      float vm[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) vm[q] = vring(m, q);  // thread-private: read before the barrier
      s_py[LV][par][wv][lane] = c3[Q - 1][1];
      __syncthreads();
      const __amdgpu_buffer_rsrc_t rx = plane_rsrc(xo, m, sz);
      float xs[Q];
      unsigned nzm = 0;   // row-compressed store: segments holding a non-zero
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        float u = vm[q];
        if (tau != 0.f) {
          const float pxm = dpp_from_left(c3[q][0]);
          const float pym = (q > 0) ? c3[q - 1][1] : s_py[LV][par][wv > 0 ? wv - 1 : 0][lane];
          float d = (xhi ? c3[q][0] : 0.f) - (xlo ? pxm : 0.f);
          d += (yhi[q] ? c3[q][1] : 0.f) - (ylo[q] ? pym : 0.f);
          if constexpr (!TV2) d += c3[q][2] - PzF(q);
          u = fmaf(tau, d, u);
        }
        if constexpr (!TV2) PzF(q) = c3[q][2];
        float xv;
        if (A.nonneg) {
          xv = fmaxf(u - A.thr, 0.f);
        } else {
          xv = copysignf(fmaxf(fabsf(u) - A.thr, 0.f), u);
        }
        xs[q] = xv;
        const bool st = zstore && ys[q];
        const bool nzr = __ballot(st && xv != 0.f) != 0;   // this wave's segment of the row holds a non-zero
        if constexpr (SP) {
          nzm |= nzr ? 1u << q : 0u;   // stored below, the wave's rows together
        } else if (zstore) {
          buf_st(rx, offs[q], xv);
        }
        if (A.rowflag != nullptr) {
          if (nzr && lane == 0) {
            A.rowflag[(size_t)m * ny + ybase + q] = 1;
            A.planeflag[m] = 1;
          }
        }
      }
      if constexpr (SP) {
        if (nzm != 0) store_rows(m, xs, nzm, zstore);
      }
      if (obj) {
        // plane m - 1 is complete now; its first rows went to slot par ^ 1
        if (m - 1 >= zb && m - 1 < ze) accumulate(xs, true, par ^ 1);
        s_x[par][wv][lane] = xs[0];  // read after the next output's barrier
#pragma unroll
        for (int q = 0; q < Q; ++q) Xp(q) = xs[q];
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
      c3[q][2] = (FIRST || TV2) ? 0.f : vcopy(P.p[q][2]);
    }
    float ppa[Q][3];   // FGP: p_prev of plane a1 (one step: output of a1 comes at the next arrival)
    if constexpr (FGP) {
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int k = 0; k < 3; ++k) ppa[q][k] = FIRST ? 0.f : vcopy(P.pp[q][k]);
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
    if constexpr (FGP) {
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int k = 0; k < 3; ++k) PPv[q][k] = ppa[q][k];
    }
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
      if (ze == nz || TV2) {
        // the last plane of the volume: no plane above it (its z-difference is
        // 0); in 2D the last plane of every chunk, which has no z margin
        __syncthreads();
        accumulate(nullptr, false, (nsteps - 1) & 1);
      }
      double s_acc = s_sum[threadIdx.x], t_acc = s_sum[NT + threadIdx.x];
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
        A.psum[blk] = s;
        A.ptv[blk] = t;
      }
    }
  }
}

// HT: tile halo, LV: fused-step register slots.  Dual passes use HT = LV = H;
// the final pass HT = H + 1, LV = H.
template <int HT, int LV, bool FINAL, bool TV2, bool FGP, bool BF, bool SP>
__device__ __forceinline__ void tv_pass_entry(const TvPassArgs& A, int bx, int by, int zb, int ze, int blk) {
  __shared__ float s_py[LV + 1][2][kTvWaves][64];  // bottom-row p_y per wave, per step (+ final), parity
  __shared__ float s_ut[LV][2][kTvWaves][64];      // top-row u per wave, per step, parity
  __shared__ float s_v[(LV + 1) * kTvQ * kTvWaves * 64];  // v ring, thread-private
  __shared__ float s_x[FINAL ? 2 : 1][kTvWaves][64];     // final pass: first-row x per wave, parity
  __shared__ double s_red[2][kTvWaves];            // final pass: per-wave sums
  __shared__ float s_fin[FINAL ? 2 * kTvQ * kTvWaves * 64 : 1];    // final pass: PzF, Xp (thread-private)
  __shared__ double s_sum[FINAL ? 2 * kTvWaves * 64 : 1];          // final pass: FP64 sums (thread-private)
  // the stop flag read once per wave (a wave-uniform branch)
  if (A.st != nullptr && __builtin_amdgcn_readfirstlane(A.st->done)) return;
  constexpr int IX = kTvRX - 2 * HT, IY = kTvRY - 2 * HT;
  const int x0 = bx * IX - HT, y0 = by * IY - HT;
  // interior tile: every point of the region and its +-1 neighbours lie inside
  const bool interior = x0 >= 1 && x0 + kTvRX <= A.nx - 1 && y0 >= 1 && y0 + kTvRY <= A.ny - 1;
  auto* sx = reinterpret_cast<float (*)[kTvWaves][64]>(&s_x[0][0][0]);
#define RIHVR_TV_BODY(E, F) \
  tv_pass_body<HT, LV, E, F, FINAL, TV2, FGP, BF, SP>(A, bx, by, zb, ze, blk, s_py, s_ut, s_v, sx, s_red, s_fin, \
                                                       s_sum)
  if (A.first) {
    if (interior) RIHVR_TV_BODY(false, true);
    else RIHVR_TV_BODY(true, true);
  } else {
    if (interior) RIHVR_TV_BODY(false, false);
    else RIHVR_TV_BODY(true, false);
  }
#undef RIHVR_TV_BODY
}

// The second launch-bounds argument is the minimum number of waves per SIMD
// the register allocation must allow: 12-wave blocks need 3 (<= 170 VGPRs,
// one block per CU), which every fusion depth fits.
constexpr int kTvWavesPerSimd = (kTvWaves + 3) / 4;

// Work of block t of a pass (t < A.nblocks): the first nfull tiles (raster
// order) times their z chunks of zchunk planes, tile-fastest; then the other
// tiles times their chunks of zchunk2 planes.
struct TvWork {
  int bx, by, zb, ze;
};
__device__ __forceinline__ TvWork tv_work(const TvPassArgs& A, uint32_t t) {
  const uint32_t n1 = (uint32_t)A.nfull * (uint32_t)((A.nz + A.zchunk - 1) / A.zchunk);
  uint32_t tile, zb, zc;
  if (t < n1) {
    tile = t % A.nfull;
    zc = A.zchunk;
    zb = (t / A.nfull) * zc;
  } else {
    const uint32_t r = (uint32_t)(A.gx * A.gy - A.nfull), u = t - n1;
    tile = A.nfull + u % r;
    zc = A.zchunk2;
    zb = (u / r) * zc;
  }
  TvWork w;
  w.bx = (int)(tile % A.gx);
  w.by = (int)(tile / A.gx);
  w.zb = (int)zb;
  w.ze = min(A.nz, (int)(zb + zc));
  return w;
}

// The first part of the grid (whole rounds of tiles) takes the XCD-contiguous
// order; the thin chunks of the split tiles, dispatched last, keep the
// hardware order so that they spread over every XCD.
template <int H, bool FINAL, bool TV2, bool FGP, bool BF, bool SP>
__global__ void __launch_bounds__(kTvWaves * 64, kTvWavesPerSimd) k_tv_pass(TvPassArgs A) {
  const uint32_t hw = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  const uint32_t n1 = (uint32_t)A.nfull * (uint32_t)((A.nz + A.zchunk - 1) / A.zchunk);
  const uint32_t t = hw < n1 ? xcd_tile(hw, n1) : hw;
  const TvWork w = tv_work(A, t);
  tv_pass_entry<FINAL ? H + 1 : H, H, FINAL, TV2, FGP, BF, SP>(A, w.bx, w.by, w.zb, w.ze, (int)t);
}

// Work item b of a batched launch: the frame f with offs[f] <= b < offs[f+1]
// and block b - offs[f] of that frame's pass.
template <int H, bool FINAL, bool TV2, bool FGP, bool BF, bool SP>
__device__ __forceinline__ void tv_batch_item(const TvPassArgs* __restrict__ args, const BatchMap& map, uint32_t b) {
  int lo = 0, hi = map.n;  // largest f with offs[f] <= b
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (map.offs[mid] <= b) lo = mid;
    else hi = mid;
  }
  lo = __builtin_amdgcn_readfirstlane(lo);  // uniform: the frame's arguments come in as scalar loads
  // read in place (scalar loads when used) rather than copied: a copy of the
  // whole struct held in scalar registers for the kernel's lifetime spills
  const TvPassArgs& A = args[lo];
  const int lb = (int)(b - (uint32_t)__builtin_amdgcn_readfirstlane(map.offs[lo]));
  const TvWork w = tv_work(A, (uint32_t)lb);
  tv_pass_entry<FINAL ? H + 1 : H, H, FINAL, TV2, FGP, BF, SP>(A, w.bx, w.by, w.zb, w.ze, lb);
}

template <int H, bool FINAL, bool TV2, bool FGP, bool BF, bool SP>
__global__ void __launch_bounds__(kTvWaves * 64, kTvWavesPerSimd) k_tv_pass_b(const TvPassArgs* __restrict__ args,
                                                                                  BatchMap map) {
  tv_batch_item<H, FINAL, TV2, FGP, BF, SP>(args, map, xcd_tile(blockIdx.x, gridDim.x));
}

// Persistent form of the batched pass: a grid of about one block per compute
// unit takes the launch's work items (every frame's blocks end to end, as
// above) from a device queue instead of running one item per block.  The items
// are cut into one contiguous range per XCD, each with a claim counter; a
// block claims items one at a time with an atomic add, from its own XCD's
// range first (neighbouring tiles share that XCD's L2), then from the other
// ranges in turn, so that the blocks that run out of work early take over the
// tail.  Items are independent and a block runs one whole item between two
// barriers, so the results do not depend on which block ran which item.  The
// last block out resets the counters: the next launch, a graph replay
// included, finds them at zero.
// The claim takes no branch on the thread index: every thread adds to the
// counter (thread 0 one, the others zero) and to the LDS word (thread 0 its
// claim, the others zero).  A branch on thread 0 here, next to the final
// pass's own thread-0 epilogue at the end of an item, lets the compiler thread
// the two across the loop's back edge and turn the item loop into an
// exec-masked loop with the barriers inside, which waves leave after
// different numbers of trips.
template <int H, bool FINAL, bool TV2, bool FGP, bool BF, bool SP>
__global__ void __launch_bounds__(kTvWaves * 64, kTvWavesPerSimd) k_tv_pass_q(const TvPassArgs* __restrict__ args,
                                                                                  BatchMap map) {
  __shared__ uint32_t s_item;
  const uint32_t n = __builtin_amdgcn_readfirstlane(map.offs[map.n]);
  const uint32_t q = n / kXcds, r = n % kXcds, home = blockIdx.x % kXcds;
  const uint32_t one = threadIdx.x == 0 ? 1u : 0u;
  s_item = 0u;
  __syncthreads();
  for (uint32_t j = 0; j < kXcds; ++j) {
    const uint32_t k = (home + j) % kXcds;
    const uint32_t first = k * q + min(k, r), len = q + (k < r ? 1u : 0u);
    for (;;) {
      const uint32_t c = atomicAdd(map.queue + k * kQueueStride, one);
      atomicAdd(&s_item, one * c);
      __syncthreads();
      const uint32_t i = __builtin_amdgcn_readfirstlane(s_item);
      __syncthreads();  // every wave holds the item before the word is cleared
      s_item = 0u;
      __syncthreads();  // ... and cleared before the next claim adds to it
      if (i >= len) break;
      tv_batch_item<H, FINAL, TV2, FGP, BF, SP>(args, map, first + i);
    }
  }
  // every block passes here once, after its last claim on every counter
  if (threadIdx.x == 0 && atomicAdd(map.queue + kXcds * kQueueStride, 1u) == gridDim.x - 1)
    for (uint32_t k = 0; k <= kXcds; ++k) atomicExch(map.queue + k * kQueueStride, 0u);
}

template <int H, bool FINAL, bool TV2, bool FGP, bool BF, bool SP>
static void launch_batched(dim3 g, const TvPassArgs* a, const BatchMap& map, hipStream_t s) {
  const dim3 b(kTvWaves * 64);
  if (map.queue != nullptr)
    hipLaunchKernelGGL((k_tv_pass_q<H, FINAL, TV2, FGP, BF, SP>), dim3(std::max(1, std::min<int>(g.x, map.grid))), b,
                       0, s, a, map);
  else hipLaunchKernelGGL((k_tv_pass_b<H, FINAL, TV2, FGP, BF, SP>), g, b, 0, s, a, map);
}

// Blocks of one pass: x tiles, y tiles, z chunks.  The z-range is cut into
// chunks of at least 16 planes until the grid holds about `want` blocks.
// `halo` is the tile halo of the pass (H on dual passes, H + 1 on the final).
struct TvGrid {
  int gx, gy, zchunk, nfull, zchunk2, nblocks;
};

static TvGrid pass_grid(int nx, int ny, int nz, int halo, int want) {
  TvGrid g{};
  g.gx = (nx + (kTvRX - 2 * halo) - 1) / (kTvRX - 2 * halo);
  g.gy = (ny + (kTvRY - 2 * halo) - 1) / (kTvRY - 2 * halo);
  const int tiles = g.gx * g.gy;
  const int nzc = std::max(1, std::min(nz / 16, (want + tiles - 1) / tiles));
  g.zchunk = (nz + nzc - 1) / nzc;
  g.nfull = tiles;
  g.zchunk2 = g.zchunk;
  g.nblocks = tiles * ((nz + g.zchunk - 1) / g.zchunk);
  return g;
}

// The final pass runs one 12-wave block per compute unit, so its time is
// whole rounds of `cus` blocks.  Its tiles are one voxel smaller than those of
// the dual passes; when they fill whole rounds but for a few (at 1024^2 one
// tile beyond 512), the leftover tiles are cut into thin z chunks that run
// side by side in one short extra round instead of a full one.
static TvGrid final_grid(int nx, int ny, int nz, int H, int want, int cus) {
  TvGrid g = pass_grid(nx, ny, nz, H + 1, want);
  const int tiles = g.gx * g.gy;
  if (cus <= 0 || g.zchunk < nz || tiles <= cus) return g;
  const int r = tiles % cus;
  const int k = r > 0 ? std::min(nz, cus / r) : 1;
  if (k < 2) return g;
  g.nfull = tiles - r;
  g.zchunk2 = (nz + k - 1) / k;
  g.nblocks = g.nfull + r * ((nz + g.zchunk2 - 1) / g.zchunk2);
  return g;
}

static int clamp_levels(int H) { return H < kTvLevelsMin ? kTvDefaultLevels : std::min(H, kTvLevelsMax); }

int prox_passes(int inner_iters, double tau, int levels, bool fgp) {
  if (!(tau > 0.0) || inner_iters <= 0) return 1;
  if (fgp) return inner_iters;        // one accelerated step per pass
  const int H = clamp_levels(levels);
  return (inner_iters + H - 1) / H;   // H dual steps per pass, the final pass included
}

// Fusion depth a prox runs with (FGP passes use the depth-2 tiles).
int prox_levels(int levels, bool fgp) { return fgp ? 2 : clamp_levels(levels); }

size_t tv_pass_args_size() { return sizeof(TvPassArgs); }

int tv_pass_blocks(int nx, int ny, int nz, int levels, int blocks) {
  return pass_grid(nx, ny, nz, clamp_levels(levels), blocks > 0 ? blocks : kTvDefaultBlocks).nblocks;
}

int tv_final_blocks(int nx, int ny, int nz, int levels, int blocks, int cus) {
  return final_grid(nx, ny, nz, clamp_levels(levels), blocks > 0 ? blocks : kTvDefaultBlocks, cus).nblocks;
}

int tv_blocks_bound(int nx, int ny, int nz, int cus) {
  // the most tiles (the final pass's halo at the deepest fusion) times the
  // most z chunks pass_grid makes, or the split of final_grid (at most one
  // thin chunk per compute unit beyond the tiles)
  const int h = kTvLevelsMax + 1;
  const int tx = (nx + (kTvRX - 2 * h) - 1) / (kTvRX - 2 * h);
  const int ty = (ny + (kTvRY - 2 * h) - 1) / (kTvRY - 2 * h);
  return tx * ty * std::max(1, nz / 16) + std::max(cus, 0);
}

int tv_group_final_blocks(int nx, int ny, int nz, int G, int levels, int blocks, int cus) {
  int total = 0;
  for (int z0 = 0; z0 < nz; z0 += G) total += tv_final_blocks(nx, ny, std::min(G, nz - z0), levels, blocks, cus);
  return total;
}

int tv_group_blocks_bound(int nx, int ny, int nz, int G, int cus) {
  const int groups = (nz + G - 1) / G;
  return groups * tv_blocks_bound(nx, ny, std::min(G, nz), cus);
}

int tv_pass_zchunk(int nx, int ny, int nz, int levels, int blocks) {
  return pass_grid(nx, ny, nz, clamp_levels(levels), blocks > 0 ? blocks : kTvDefaultBlocks).zchunk;
}

// Argument structs of every pass of one prox application.  Every pass takes
// up to H dual steps; the final pass (its own tile grid, halo H + 1) also
// recovers the primal, thresholds and stores x.
int prox_pass_args(const ProxArgs& pa, void* out, int* blocks_per_pass) {
  const double tau = pa.step * pa.tv;
  const double thr = pa.step * pa.l1;
  const bool use_tv = tau > 0.0 && pa.inner_iters > 0;
  const int K = use_tv ? pa.inner_iters : 0;
  const bool fgp = pa.fgp != 0;
  const int H = prox_levels(pa.levels, fgp);
  const int npass = prox_passes(K, tau, H, fgp);
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
  a.tv2 = pa.tv2 ? 1 : 0;
  a.dual_bf16 = pa.dual_bf16 ? 1 : 0;
  a.rs = pa.rs;
  a.c = use_tv ? (float)(1.0 / ((pa.tv2 ? 8.0 : 12.0) * tau)) : 0.f;
  a.thr = (float)thr;
  const int want = pa.blocks > 0 ? pa.blocks : kTvDefaultBlocks;
  TvPassArgs* o = static_cast<TvPassArgs*>(out);
  int done = 0;
  double tk = 1.0;   // FGP: t_k of the step a pass takes
  for (int p = 0; p < npass; ++p) {
    const bool fin = p == npass - 1;
    const TvGrid g = fin ? final_grid(pa.nx, pa.ny, pa.nz, H, want, pa.cus) : pass_grid(pa.nx, pa.ny, pa.nz, H, want);
    a.gx = g.gx;
    a.gy = g.gy;
    a.zchunk = g.zchunk;
    a.nfull = g.nfull;
    a.zchunk2 = g.zchunk2;
    a.nblocks = g.nblocks;
    if (blocks_per_pass) blocks_per_pass[p] = g.nblocks;
    const int lv = fgp ? std::min(1, K - done) : std::min(H, K - done);
    a.levels = lv;
    a.first = (done == 0 && !pa.warm) ? 1 : 0;   // a warm dual is read by the first pass
    a.final_ = fin ? 1 : 0;
    a.keep_dual = (fin && pa.warm) ? 1 : 0;
    a.flip_npass = (pa.warm && (npass & 1)) ? npass : 0;
    a.fgp = (fgp && !fin) ? 1 : 0;
    const double tn = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * tk * tk));
    a.fgp_w = (float)((tk - 1.0) / tn);
    tk = tn;
    float* const* src = (p & 1) ? pa.pb : pa.pa;
    float* const* dst = (p & 1) ? pa.pa : pa.pb;
    float* const* src2 = (p & 1) ? pa.pb2 : pa.pa2;
    float* const* dst2 = (p & 1) ? pa.pa2 : pa.pb2;
    for (int k = 0; k < 3; ++k) {
      const bool none = pa.tv2 && k == 2;
      a.pin[k] = none ? nullptr : src[k];
      a.pout[k] = none ? nullptr : dst[k];
      a.pin2[k] = (none || !fgp) ? nullptr : src2[k];
      a.pout2[k] = (none || !fgp) ? nullptr : dst2[k];
    }
    o[p] = a;
    done += lv;
  }
  return npass;
}

// Kernel selection: fusion depth, final / dual pass, 2D or 3D TV, FGP (dual
// passes of depth-2 tiles only), bfloat16 dual, row-compressed output (final
// passes with an FP32 dual only).  BATCH picks the batched form.
template <bool BATCH, bool FINAL, bool TV2, bool FGP, bool BF, bool SP>
static void launch_k(int H, dim3 g, const TvPassArgs* a, BatchMap map, hipStream_t s) {
  const dim3 b(kTvWaves * 64);
  if constexpr (FGP) {
    if constexpr (BATCH) launch_batched<2, FINAL, TV2, true, BF, false>(g, a, map, s);
    else hipLaunchKernelGGL((k_tv_pass<2, FINAL, TV2, true, BF, false>), g, b, 0, s, *a);
  } else {
    switch (H) {
      case 2:
        if constexpr (BATCH) launch_batched<2, FINAL, TV2, false, BF, SP>(g, a, map, s);
        else hipLaunchKernelGGL((k_tv_pass<2, FINAL, TV2, false, BF, SP>), g, b, 0, s, *a);
        break;
      case 3:
        if constexpr (BATCH) launch_batched<3, FINAL, TV2, false, BF, SP>(g, a, map, s);
        else hipLaunchKernelGGL((k_tv_pass<3, FINAL, TV2, false, BF, SP>), g, b, 0, s, *a);
        break;
      default:
        if constexpr (BATCH) launch_batched<4, FINAL, TV2, false, BF, SP>(g, a, map, s);
        else hipLaunchKernelGGL((k_tv_pass<4, FINAL, TV2, false, BF, SP>), g, b, 0, s, *a);
        break;
    }
  }
}

template <bool BATCH, bool FINAL, bool TV2>
static void launch_sel(bool fgp, bool bf, bool sp, int H, dim3 g, const TvPassArgs* a, BatchMap map,
                       hipStream_t s) {
  if constexpr (!FINAL) {
    if (fgp) {
      if (bf) launch_k<BATCH, false, TV2, true, true, false>(H, g, a, map, s);
      else launch_k<BATCH, false, TV2, true, false, false>(H, g, a, map, s);
      return;
    }
  } else {
    if (sp && !bf) {
      launch_k<BATCH, true, TV2, false, false, true>(H, g, a, map, s);
      return;
    }
  }
  if (bf) launch_k<BATCH, FINAL, TV2, false, true, false>(H, g, a, map, s);
  else launch_k<BATCH, FINAL, TV2, false, false, false>(H, g, a, map, s);
}

template <bool BATCH>
static void launch_any(bool final_pass, bool tv2, bool fgp, bool bf, bool sp, int H, dim3 g, const TvPassArgs* a,
                       BatchMap map, hipStream_t s) {
  if (final_pass) {
    if (tv2) launch_sel<BATCH, true, true>(false, bf, sp, H, g, a, map, s);
    else launch_sel<BATCH, true, false>(false, bf, sp, H, g, a, map, s);
  } else {
    if (tv2) launch_sel<BATCH, false, true>(fgp, bf, false, H, g, a, map, s);
    else launch_sel<BATCH, false, false>(fgp, bf, false, H, g, a, map, s);
  }
}

// The per-plane 2D TV couples no planes, so its prox can run on groups of G
// planes in turn, each group's passes reading and writing a dual of G planes
// (the paper's plane-by-plane prox, with the memory of G planes instead of the
// volume).  Each group's final pass writes its objective partials after the
// previous groups' ones.
static hipError_t launch_prox_grouped(const ProxArgs& pa, int K, int H, int np, hipStream_t s, int* launches) {
  const int G = pa.group_planes;
  const size_t plane = (size_t)pa.nx * pa.ny;
  std::vector<TvPassArgs> args(np);
  std::vector<int> nb(np);
  int off = 0, nl = 0;
  for (int z0 = 0; z0 < pa.nz; z0 += G) {
    ProxArgs q = pa;
    q.nz = std::min(G, pa.nz - z0);
    q.group_planes = 0;
    q.rowflag = pa.rowflag ? pa.rowflag + (size_t)z0 * pa.ny : nullptr;
    q.planeflag = pa.planeflag ? pa.planeflag + z0 : nullptr;
    q.psum = pa.psum ? pa.psum + off : nullptr;
    q.ptv = pa.ptv ? pa.ptv + off : nullptr;
    if (pa.stage_group) q.x = pa.stage_group;
    const int npass = prox_pass_args(q, args.data(), nb.data());
    for (int p = 0; p < npass; ++p) {
      args[p].zoff_v = (size_t)z0 * plane;
      args[p].zoff_x = pa.stage_group ? 0 : (size_t)z0 * plane;
      launch_any<false>(args[p].final_ != 0, args[p].tv2 != 0, args[p].fgp != 0, args[p].dual_bf16 != 0,
                        args[p].rs.on != 0, H, dim3(nb[p]), &args[p], BatchMap{nullptr, 0}, s);
    }
    nl += npass;
    if (pa.stage_group) {
      const hipError_t e = launch_copy_f32(pa.x + (size_t)z0 * plane, pa.stage_group, (size_t)q.nz * plane, s);
      if (e != hipSuccess) return e;
      ++nl;
    }
    off += nb[npass - 1];
  }
  if (launches) *launches = nl;
  return hipGetLastError();
}

hipError_t launch_prox(const ProxArgs& pa, hipStream_t s, int* launches) {
  const double tau = pa.step * pa.tv;
  const int K = (tau > 0.0 && pa.inner_iters > 0) ? pa.inner_iters : 0;
  const int H = prox_levels(pa.levels, pa.fgp != 0);
  const int np = prox_passes(K, tau, H, pa.fgp != 0);
  if (pa.tv2 && pa.group_planes > 0 && pa.group_planes < pa.nz) return launch_prox_grouped(pa, K, H, np, s, launches);
  std::vector<TvPassArgs> args(np);
  std::vector<int> nb(np);
  const int npass = prox_pass_args(pa, args.data(), nb.data());
  for (int p = 0; p < npass; ++p)
    launch_any<false>(args[p].final_ != 0, args[p].tv2 != 0, args[p].fgp != 0, args[p].dual_bf16 != 0,
                      args[p].rs.on != 0, H, dim3(nb[p]), &args[p], BatchMap{nullptr, 0}, s);
  if (launches) *launches = npass;
  return hipGetLastError();
}

hipError_t launch_tv_pass_batched(int levels, bool final_pass, bool tv2, bool fgp, bool bf16, bool sparse,
                                  const void* args, BatchMap map, int nblocks, hipStream_t s) {
  launch_any<true>(final_pass, tv2, fgp && !final_pass, bf16, sparse, clamp_levels(levels), dim3(nblocks),
                   static_cast<const TvPassArgs*>(args), map, s);
  return hipGetLastError();
}

}  // namespace rihvr
