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
// block owns a 64 x (8 Q) tile in (x, y) -- one wavefront lane per x, Q rows of
// y per lane, 8 wavefronts stacked in y -- and streams through z.  The L steps
// form a pipeline along z: step l consumes the dual of step l-1 one plane
// behind it and keeps in registers, per point, the previous plane's dual and
// primal values.  Neighbours along x move with DPP wave shifts, along y through
// registers within a lane and through double-buffered LDS rows between
// wavefronts (one barrier per step and plane).  Points within L of the tile
// edge are computed but not stored; tiles overlap by 2L.  The z-range is cut
// into chunks with an L+1 plane margin so that the grid fills the device.
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

constexpr int kTvWaves = 8;
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
  const SolveState* st;
  int nx, ny, nz;
  int levels;                     // fused dual steps in this pass (<= H, <= H-1 when final)
  int first, final_, nonneg;
  int zchunk;                     // output planes per block
  float tau, c, thr;
  int gx, gy;                     // tiles along x and y (the grid of one frame)
};

__device__ __forceinline__ float dpp_from_left(float v) {   // lane i <- lane i-1 (0 at lane 0)
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float dpp_from_right(float v) {  // lane i <- lane i+1 (0 at lane 63)
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xf, 0xf, true));
}

// Pass body.  EDGE: the tile touches the volume boundary, so every access and
// every difference is masked; interior tiles (most of them) skip the masks.
// FIRST: the incoming dual is zero (nothing is read).
// A pointer known to be the same in every lane (keeps address bases in SGPRs).
template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  const uint64_t u = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
  return reinterpret_cast<T*>(((uint64_t)hi << 32) | lo);
}

template <int H, bool EDGE, bool FIRST>
__device__ __forceinline__ void tv_pass_body(const TvPassArgs& A, int bx, int by, int bz,
                                             float (*s_py)[2][kTvWaves][64], float (*s_ut)[2][kTvWaves][64],
                                             float* s_v) {
  constexpr int Q = kTvQ, NW = kTvWaves, NT = NW * 64;
  constexpr int IX = kTvRX - 2 * H, IY = kTvRY - 2 * H;  // interior (stored) extent
  const float* __restrict__ v = uniform_ptr(A.v ? A.v : A.vol[A.st->prev]);
  float* __restrict__ xo = uniform_ptr(A.x ? A.x : A.vol[A.st->next]);
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

  bool iny[Q], ylo[Q], yhi[Q], ys[Q];
  unsigned off[Q];  // in-plane byte offset (32 bit, so loads use a scalar base + vector offset)
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int y = ybase + q;
    iny[q] = !EDGE || (y >= 0 && y < ny);
    ylo[q] = !EDGE || y > 0;
    yhi[q] = !EDGE || y + 1 < ny;
    const int r = wv * Q + q;
    ys[q] = iny[q] && r >= H && r < kTvRY - H;
    off[q] = (inx && iny[q]) ? (unsigned)(y * nx + x) * 4u : 0u;
  }
  // per fused step: previous plane's dual (3) and primal (1); final stage: previous p_z
  float Pp[H][Q][3], Up[H][Q], PzF[Q];
#pragma unroll
  for (int l = 0; l < H; ++l)
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      Pp[l][q][0] = Pp[l][q][1] = Pp[l][q][2] = 0.f;
      Up[l][q] = 0.f;
    }
#pragma unroll
  for (int q = 0; q < Q; ++q) PzF[q] = 0.f;

  // v of recent planes lives in a thread-private LDS ring (slot = plane mod H+1);
  // the next plane's v and dual are prefetched into registers one step ahead.
  float vN[Q], pN[Q][3];
  auto ld = [](const float* base, unsigned ob) -> float {
    return *(const __attribute__((address_space(1))) float*)(reinterpret_cast<const char*>(base) + ob);
  };
  auto load_plane = [&](int a) {
    const float* vp = v + (size_t)a * sz;
#pragma unroll
    for (int q = 0; q < Q; ++q) vN[q] = (inx && iny[q]) ? ld(vp, off[q]) : 0.f;
    if constexpr (!FIRST) {
      const float* p0 = A.pin[0] + (size_t)a * sz;
      const float* p1 = A.pin[1] + (size_t)a * sz;
      const float* p2 = A.pin[2] + (size_t)a * sz;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const bool in = inx && iny[q];
        pN[q][0] = in ? ld(p0, off[q]) : 0.f;
        pN[q][1] = in ? ld(p1, off[q]) : 0.f;
        pN[q][2] = in ? ld(p2, off[q]) : 0.f;
      }
    }
  };
  auto st_ = [](float* base, unsigned ob, float val) {
    *(__attribute__((address_space(1))) float*)(reinterpret_cast<char*>(base) + ob) = val;
  };
  if constexpr (FIRST) {
#pragma unroll
    for (int q = 0; q < Q; ++q) pN[q][0] = pN[q][1] = pN[q][2] = 0.f;
  }
  auto vring = [&](int a, int q) -> float& { return s_v[((a % (H + 1)) * Q + q) * NT + threadIdx.x]; };
  load_plane(zs);

  const int nsteps = (zl - zs) + L;
  for (int s = 0; s < nsteps; ++s) {
    const int par = s & 1;
    const int a1 = zs + s;
    float c3[Q][3];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      if (a1 < zl) vring(a1, q) = vN[q];
      c3[q][0] = pN[q][0];
      c3[q][1] = pN[q][1];
      c3[q][2] = pN[q][2];
    }
    if (a1 + 1 < zl) load_plane(a1 + 1);
#pragma unroll
    for (int l = 0; l < H; ++l) {
      if (l >= L) break;
      const int a = zs + s - l;          // arrival plane of fused step l
      if (a < zs || a > zl) continue;    // idle (uniform across the block)
      if (a < zl) {
        // ---- arrival of the previous dual at plane a ----
        s_py[l][par][wv][lane] = c3[Q - 1][1];
        __syncthreads();
        float un[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const float pxm = dpp_from_left(c3[q][0]);
          const float pym = (q > 0) ? c3[q - 1][1] : s_py[l][par][wv > 0 ? wv - 1 : 0][lane];
          float d = (xhi ? c3[q][0] : 0.f) - (xlo ? pxm : 0.f);
          d += (yhi[q] ? c3[q][1] : 0.f) - (ylo[q] ? pym : 0.f);
          d += c3[q][2] - Pp[l][q][2];
          un[q] = fmaf(tau, d, vring(a, q));
        }
        if (a > zs) {
          // ---- dual step at plane a - 1 ----
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
      } else {
        // ---- flush: dual step at the last plane zl - 1 (no plane above) ----
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
      }
    }
    // ---- output stage: dual of the last fused step at plane m = zs + s - L ----
    const int m = zs + s - L;
    if (m < zs || m >= zl) continue;
    const bool zstore = m >= zb && m < ze;
    if (!A.final_) {
      if (zstore && ix_store) {
        float* o0 = A.pout[0] + (size_t)m * sz;
        float* o1 = A.pout[1] + (size_t)m * sz;
        float* o2 = A.pout[2] + (size_t)m * sz;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          if (!ys[q]) continue;
          st_(o0, off[q], c3[q][0]);
          st_(o1, off[q], c3[q][1]);
          st_(o2, off[q], c3[q][2]);
        }
      }
    } else {
      // primal recovery u = v + tau div p, soft threshold, store, flags
      s_py[H][par][wv][lane] = c3[Q - 1][1];
      __syncthreads();
      float* xp = xo + (size_t)m * sz;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        float u = vring(m, q);
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
        const bool st = zstore && ix_store && ys[q];
        if (st) st_(xp, off[q], xv);
        if (A.rowflag != nullptr) {
          const bool nzr = __ballot(st && xv != 0.f) != 0;
          if (nzr && lane == 0) {
            A.rowflag[(size_t)m * ny + ybase + q] = 1;
            A.planeflag[m] = 1;
          }
        }
      }
    }
  }
}

template <int H>
__device__ __forceinline__ void tv_pass_entry(const TvPassArgs& A, int bx, int by, int bz) {
  __shared__ float s_py[H + 1][2][kTvWaves][64];  // bottom-row p_y per wave, per step, parity
  __shared__ float s_ut[H][2][kTvWaves][64];      // top-row u per wave, per step, parity
  __shared__ float s_v[(H + 1) * kTvQ * kTvWaves * 64];  // v ring, thread-private
  if (A.st != nullptr && A.st->done) return;
  constexpr int IX = kTvRX - 2 * H, IY = kTvRY - 2 * H;
  const int x0 = bx * IX - H, y0 = by * IY - H;
  // interior tile: every point of the region and its +-1 neighbours lie inside
  const bool interior = x0 >= 1 && x0 + kTvRX <= A.nx - 1 && y0 >= 1 && y0 + kTvRY <= A.ny - 1;
  if (A.first) {
    if (interior) tv_pass_body<H, false, true>(A, bx, by, bz, s_py, s_ut, s_v);
    else tv_pass_body<H, true, true>(A, bx, by, bz, s_py, s_ut, s_v);
  } else {
    if (interior) tv_pass_body<H, false, false>(A, bx, by, bz, s_py, s_ut, s_v);
    else tv_pass_body<H, true, false>(A, bx, by, bz, s_py, s_ut, s_v);
  }
}

// Register budget: the two- and three-deep pipelines fit 128 VGPRs, so LDS
// (not registers) limits them to two blocks of eight waves per CU; the
// four-deep one, and the three-deep batched entry (which also holds the frame
// lookup), keep their full register file.
template <int H, bool BATCHED>
constexpr int tv_min_blocks() { return (H <= 2 || (H == 3 && !BATCHED)) ? 4 : 1; }

template <int H>
__global__ void __launch_bounds__(kTvWaves * 64, (tv_min_blocks<H, false>())) k_tv_pass(TvPassArgs A) {
  tv_pass_entry<H>(A, blockIdx.x, blockIdx.y, blockIdx.z);
}

template <int H>
__global__ void __launch_bounds__(kTvWaves * 64, (tv_min_blocks<H, true>())) k_tv_pass_b(const TvPassArgs* __restrict__ args,
                                                                                  BatchMap map) {
  const uint32_t b = blockIdx.x;
  int lo = 0, hi = map.n;  // largest f with offs[f] <= b
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (map.offs[mid] <= b) lo = mid;
    else hi = mid;
  }
  const TvPassArgs A = args[lo];
  const int lb = (int)(b - map.offs[lo]);
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
