// Warm-start 3D U-Net kernels for gfx950: BF16 activations and weights, FP32
// accumulation on the matrix cores (v_mfma_f32_16x16x32_bf16).
//
// Activations are channels-last, [z][y][x][c] with a channel stride (so a
// concatenation is two views of one buffer).  Every convolution-like layer is
// one "gather GEMM": row r is an output voxel, the reduction index k = t*C + c
// runs over taps t and input channels c, and the operand row of tap t is read
// from a source voxel chosen by the layer's gather mode.  Weights are packed as
// B[t][n][c] (n the GEMM column, c contiguous) so each lane loads 8 consecutive
// reduction values with one 16-byte load.
//
// MFMA 16x16x32 operand layout (per wavefront of 64 lanes, lane l):
//   A (16 x 32): row l % 16, reduction elements 8 (l / 16) .. 8 (l / 16) + 7
//   B (32 x 16): column l % 16, reduction elements 8 (l / 16) .. + 7
//   D (16 x 16): rows 4 (l / 16) .. 4 (l / 16) + 3, column l % 16
#include <type_traits>

#include <cmath>

#include "unet_internal.h"

namespace rihvr {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

__device__ __forceinline__ float bf2f(uint16_t v) { return __uint_as_float((uint32_t)v << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
  // round to nearest even (finite inputs)
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// Row coordinates of one lane, computed once: the source voxel of a tap is
// then found with adds and compares only (no 64-bit division per k-step).
struct GgRow {
  int x, y, z;
  bool ok;
};
__device__ __forceinline__ GgRow gg_row(const GatherGemmArgs& a, long r, long nrows) {
  GgRow g;
  g.ok = r < nrows;
  const long rr = g.ok ? r : 0;
  const long hw = (long)a.W * a.H;
  g.z = (int)(rr / hw);
  const int rem = (int)(rr - (long)g.z * hw);
  g.y = rem / a.W;
  g.x = rem - g.y * a.W;
  return g;
}

// Source voxel (linear index at the source resolution) of a row for tap t, or -1.
template <int MODE>
__device__ __forceinline__ long gg_source_m(const GatherGemmArgs& a, const GgRow& g, int t) {
  const int D = a.D, H = a.H, W = a.W;  // row grid
  if constexpr (MODE == GG_CONV3_FWD || MODE == GG_CONV3_BWD) {
    int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;  // tap t of the 3x3x3 stencil
    if constexpr (MODE == GG_CONV3_BWD) { dz = -dz; dy = -dy; dx = -dx; }
    const int zz = g.z + dz, yy = g.y + dy, xx = g.x + dx;
    if (zz < 0 || zz >= D || yy < 0 || yy >= H || xx < 0 || xx >= W) return -1;
    return ((long)zz * H + yy) * W + xx;
  } else if constexpr (MODE == GG_UP_BWD) {
    // row (z, y, x) is a coarse voxel; tap t = dz*4 + dy*2 + dx selects the fine voxel
    const int zz = 2 * g.z + (t >> 2), yy = 2 * g.y + ((t >> 1) & 1), xx = 2 * g.x + (t & 1);
    return ((long)zz * (2 * H) + yy) * (2 * W) + xx;
  } else {  // GG_UP_FWD, GG_POINT
    return ((long)g.z * H + g.y) * W + g.x;
  }
}
__device__ __forceinline__ long gg_source(const GatherGemmArgs& a, const GgRow& g, int t) {
  switch (a.mode) {
    case GG_CONV3_FWD: return gg_source_m<GG_CONV3_FWD>(a, g, t);
    case GG_CONV3_BWD: return gg_source_m<GG_CONV3_BWD>(a, g, t);
    case GG_UP_BWD: return gg_source_m<GG_UP_BWD>(a, g, t);
    case GG_UP_FWD:
    case GG_POINT: return gg_source_m<GG_POINT>(a, g, t);
  }
  return -1;
}

// Load target of switched-off lanes (zero-initialised device memory): operand
// loads are selects of an address, never branches, so that the loads of the
// next reduction step stay in flight under the MFMAs of this one.
__device__ uint4 g_gg_zero;

// Block: 4 wavefronts x (16 RT) rows; every wavefront computes all NB column
// tiles of its RT row tiles, so a B fragment (weights) feeds RT MFMAs and an A
// fragment (gathered activations) feeds NB.  The reduction index k = t C + c
// advances by 32 per step with t, c updated incrementally.  The operands of
// step k + 32 are loaded while the MFMAs of step k run (two register sets used
// in turn; B is prefetched too while it is small).
template <int NB, int RT, int MODE>
__global__ void __launch_bounds__(256) k_gather_gemm(GatherGemmArgs a) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const long row0 = ((long)blockIdx.x * 4 + wv) * (16 * RT);
  const long nrows = (long)a.D * a.H * a.W;
  const int kq = (lane >> 4) * 8;       // reduction offset of this lane within a 32-chunk
  const int K = a.T * a.C;
  GgRow rows[RT];
#pragma unroll
  for (int i = 0; i < RT; ++i) rows[i] = gg_row(a, row0 + i * 16 + (lane & 15), nrows);
  f32x4 acc[RT][NB];
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const uint16_t* __restrict__ src = a.src + a.src_c0;
  const uint16_t* __restrict__ wt = a.wt;
  const uint4* zero = &g_gg_zero;
  constexpr bool PB = NB <= 4;   // B prefetched with A
  constexpr int NBP = PB ? NB : 1;
  struct Step {                  // operand position of one reduction step
    int t, c;
    bool kin;
  };
  auto next = [&](Step st) {
    st.c += 32;
    while (st.c >= a.C) {
      st.c -= a.C;
      ++st.t;
    }
    st.kin = st.t * a.C + st.c < K;
    return st;
  };
  // 3x3x3 modes: per row, the address of its own voxel and a mask of the taps
  // whose source voxel lies inside the grid, so that a step costs one shared
  // tap offset per lane and a bit test and an add per row
  constexpr bool CONV3 = MODE == GG_CONV3_FWD || MODE == GG_CONV3_BWD;
  constexpr int SGN = MODE == GG_CONV3_BWD ? -1 : 1;
  const uint16_t* rbase[RT];
  uint32_t tmask[RT];
  if constexpr (CONV3) {
#pragma unroll
    for (int i = 0; i < RT; ++i) {
      const GgRow& g = rows[i];
      rbase[i] = src + (((long)g.z * a.H + g.y) * a.W + g.x) * a.src_cs;
      uint32_t mz = 0, my = 0, mx = 0;  // bit d + 1 set: offset d in -1..1 stays inside
#pragma unroll
      for (int d = -1; d <= 1; ++d) {
        const int e = SGN * d;
        mz |= (g.z + e >= 0 && g.z + e < a.D) ? 1u << (d + 1) : 0u;
        my |= (g.y + e >= 0 && g.y + e < a.H) ? 1u << (d + 1) : 0u;
        mx |= (g.x + e >= 0 && g.x + e < a.W) ? 1u << (d + 1) : 0u;
      }
      uint32_t m = 0;
#pragma unroll
      for (int t = 0; t < 27; ++t)
        if (((mz >> (t / 9)) & (my >> ((t / 3) % 3)) & (mx >> (t % 3)) & 1u) != 0) m |= 1u << t;
      tmask[i] = g.ok ? m : 0u;
    }
  }
  auto tap_offset = [&](int t) -> long {  // source voxel of tap t relative to the row's voxel, in elements
    const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
    return (long)(SGN * ((dz * a.H + dy) * a.W + dx)) * a.src_cs;
  };
  auto ld_a = [&](int i, const Step& st, long toff) -> uint4 {
    if constexpr (CONV3) {
      const bool on = st.kin && ((tmask[i] >> (st.t & 31)) & 1u) != 0;   // kin implies t < 27
      return *(on ? reinterpret_cast<const uint4*>(rbase[i] + toff + st.c) : zero);
    } else {
      const long sv = gg_source_m<MODE>(a, rows[i], st.t);
      const bool on = st.kin && rows[i].ok && sv >= 0;
      return *(on ? reinterpret_cast<const uint4*>(src + sv * a.src_cs + st.c) : zero);
    }
  };
  auto ld_b = [&](int j, const Step& st) -> uint4 {
    return *(st.kin ? reinterpret_cast<const uint4*>(wt + ((size_t)st.t * a.Npad + j * 16 + (lane & 15)) * a.C + st.c)
                    : zero);
  };
  // set X holds the operands of the current step, set Y those of the next
  uint4 xa[RT], ya[RT], xb[NBP], yb[NBP];
  auto load = [&](uint4 (&sa)[RT], uint4 (&sb)[NBP], const Step& st) {
    const long toff = CONV3 ? tap_offset(st.t) : 0;
#pragma unroll
    for (int i = 0; i < RT; ++i) sa[i] = ld_a(i, st, toff);
    if constexpr (PB) {
#pragma unroll
      for (int j = 0; j < NB; ++j) sb[j] = ld_b(j, st);
    }
  };
  auto mma = [&](const uint4 (&sa)[RT], const uint4 (&sb)[NBP], const Step& st) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const bf16x8 bv = __builtin_bit_cast(bf16x8, PB ? sb[j] : ld_b(j, st));
#pragma unroll
      for (int i = 0; i < RT; ++i)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, sa[i]), bv, acc[i][j], 0, 0, 0);
    }
  };
  Step cur{kq / a.C, kq - (kq / a.C) * a.C, kq < K};
  load(xa, xb, cur);
  // two steps per trip; a trailing step past K reads zeros and adds nothing
  for (int k0 = 0; k0 < K; k0 += 64) {
    const Step s1 = next(cur);
    load(ya, yb, s1);
    mma(xa, xb, cur);
    const Step s2 = next(s1);
    load(xa, xb, s2);
    mma(ya, yb, s1);
    cur = s2;
  }
  // epilogue: rows 4 (lane / 16) + i of each row tile, column 16 j + lane % 16
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int n = j * 16 + (lane & 15);
      if (n >= a.N) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const long r = row0 + rt * 16 + (lane >> 4) * 4 + i;
        if (r >= nrows) continue;
        float v = acc[rt][j][i];
        long dvox = r;
        int dch = n;
        if (a.mode == GG_UP_FWD) {
          // column n = d * Cout + co writes fine voxel 2 q + d, channel co
          const int d = n / a.up_cout, co = n - d * a.up_cout;
          const GgRow g = gg_row(a, r, nrows);
          dvox = ((long)(2 * g.z + (d >> 2)) * (2 * a.H) + 2 * g.y + ((d >> 1) & 1)) * (2 * a.W) + 2 * g.x + (d & 1);
          dch = co;
        }
        if (a.bias) v += a.bias[dch];
        if (a.relu) v = fmaxf(v, 0.f);
        const size_t o = (size_t)dvox * a.dst_cs + a.dst_c0 + dch;
        if (a.out_f32) {
          float* d = reinterpret_cast<float*>(a.dst);
          d[o] = a.accumulate ? d[o] + v : v;
        } else {
          uint16_t* d = reinterpret_cast<uint16_t*>(a.dst);
          d[o] = f2bf(a.accumulate ? bf2f(d[o]) + v : v);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// 3x3x3 layers from an LDS halo tile.  A block's rows are a 16 x 4 x RT box of
// output voxels (x fastest; wavefront w takes y0 + w, row tile i takes z0 + i,
// MFMA row m takes x0 + m).  The input box with a one-voxel halo, 18 x 6 x
// (RT + 2) voxels of all C channels with zeros outside the grid, is staged in
// LDS once, and every tap reads its A operand there at a fixed offset, instead
// of gathering it from global memory nine to 27 times per voxel.
// ---------------------------------------------------------------------------
constexpr int kHbX = 18, kHbY = 6;  // halo box extent in x and y

template <int NB, int RT, int MODE>
__global__ void __launch_bounds__(256) k_conv3_lds(GatherGemmArgs a) {
  extern __shared__ uint4 s_box4[];
  uint16_t* s_box = reinterpret_cast<uint16_t*>(s_box4);  // [RT + 2][6][18][C]
  constexpr int BZ = RT + 2;
  constexpr int SGN = MODE == GG_CONV3_BWD ? -1 : 1;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int C = a.C;
  const int x0 = blockIdx.x * 16, y0 = blockIdx.y * 4, z0 = blockIdx.z * RT;
  const int cch = C / 8;  // 16-byte chunks per voxel
  const int nchunk = kHbX * kHbY * BZ * cch;
  for (int e = threadIdx.x; e < nchunk; e += 256) {
    const int v = e / cch, q = e - v * cch;
    const int bx = v % kHbX, by = (v / kHbX) % kHbY, bz = v / (kHbX * kHbY);
    const int gx = x0 + bx - 1, gy = y0 + by - 1, gz = z0 + bz - 1;
    uint4 val = make_uint4(0, 0, 0, 0);
    if (gx >= 0 && gx < a.W && gy >= 0 && gy < a.H && gz >= 0 && gz < a.D)
      val = *reinterpret_cast<const uint4*>(a.src + (((long)gz * a.H + gy) * a.W + gx) * a.src_cs + a.src_c0 +
                                            q * 8);
    s_box4[e] = val;  // chunk e is voxel v, channels 8q .. 8q + 7
  }
  __syncthreads();
  const int lx = lane & 15;
  const int kq = (lane >> 4) * 8;
  const int K = 27 * C;
  const uint16_t* __restrict__ wt = a.wt;
  const uint4* zero = &g_gg_zero;
  f32x4 acc[RT][NB];
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  // the weights of step k + 32 are loaded while the MFMAs of step k run (two
  // register sets used in turn); a trailing step past K reads zeros
  struct Step {
    int t, c;
    bool kin;
  };
  auto next = [&](Step st) {
    st.c += 32;
    while (st.c >= C) {
      st.c -= C;
      ++st.t;
    }
    st.kin = st.t * C + st.c < K;  // t < 27
    return st;
  };
  auto ld_b = [&](uint4 (&sb)[NB], const Step& st) {
#pragma unroll
    for (int j = 0; j < NB; ++j)
      sb[j] = *(st.kin ? reinterpret_cast<const uint4*>(wt + ((size_t)st.t * a.Npad + j * 16 + lx) * C + st.c) : zero);
  };
  auto mma = [&](const uint4 (&sb)[NB], const Step& st) {
    const int tt = st.kin ? st.t : 13;  // the centre tap keeps the LDS index inside the box
    const int dz = SGN * (tt / 9 - 1), dy = SGN * ((tt / 3) % 3 - 1), dx = SGN * (tt % 3 - 1);
    bf16x8 av[RT];
#pragma unroll
    for (int i = 0; i < RT; ++i) {
      const int vi = ((i + 1 + dz) * kHbY + (wv + 1 + dy)) * kHbX + (lx + 1 + dx);
      const uint4 raw = *reinterpret_cast<const uint4*>(s_box + (size_t)vi * C + st.c);
      av[i] = __builtin_bit_cast(bf16x8, st.kin ? raw : make_uint4(0, 0, 0, 0));
    }
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const bf16x8 bv = __builtin_bit_cast(bf16x8, sb[j]);
#pragma unroll
      for (int i = 0; i < RT; ++i) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv, acc[i][j], 0, 0, 0);
    }
  };
  uint4 xb[NB], yb[NB];
  Step cur{kq / C, kq - (kq / C) * C, kq < K};
  ld_b(xb, cur);
  for (int k0 = 0; k0 < K; k0 += 64) {
    const Step s1 = next(cur);
    ld_b(yb, s1);
    mma(xb, cur);
    const Step s2 = next(s1);
    ld_b(xb, s2);
    mma(yb, s1);
    cur = s2;
  }
  // epilogue: D row m = 4 (lane / 16) + i is voxel (x0 + m, y0 + wv, z0 + rt)
  const int y = y0 + wv;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int z = z0 + rt;
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const int n = j * 16 + lx;
      if (n >= a.N) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int x = x0 + (lane >> 4) * 4 + i;
        if (x >= a.W || y >= a.H || z >= a.D) continue;
        float v = acc[rt][j][i];
        if (a.bias) v += a.bias[n];
        if (a.relu) v = fmaxf(v, 0.f);
        const size_t o = (size_t)(((long)z * a.H + y) * a.W + x) * a.dst_cs + a.dst_c0 + n;
        if (a.out_f32) {
          float* d = reinterpret_cast<float*>(a.dst);
          d[o] = a.accumulate ? d[o] + v : v;
        } else {
          uint16_t* d = reinterpret_cast<uint16_t*>(a.dst);
          d[o] = f2bf(a.accumulate ? bf2f(d[o]) + v : v);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Weight gradient: dW[t][c][n] += sum_r S(r, t)[c] * G(r, t)[n]  (FP32 atomics;
// [t][c][n] is the [tap][cin][cout] layout of the master weights).
// Block: one tap, a chunk of rows and a group of up to 16 (n, c) output tiles;
// 32-row slabs of G and S are staged in LDS, tiles are spread over the 4
// wavefronts.
// ---------------------------------------------------------------------------
constexpr int kWgRows = 32;
constexpr int kWgMaxN = 128, kWgMaxC = 256;

__global__ void __launch_bounds__(256) k_wgrad(WgradArgs a) {
  __shared__ uint16_t sg[kWgRows][kWgMaxN];
  __shared__ uint16_t ss[kWgRows][kWgMaxC];
  const int t = blockIdx.y;
  const long nrows = (long)a.D * a.H * a.W;
  const long r0 = (long)blockIdx.x * a.rows_per_block;
  const long r1 = min(nrows, r0 + a.rows_per_block);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int tn = a.Npad / 16, tc = a.Cpad / 16, ntile = tn * tc;
  constexpr int MAXT = 4;  // tiles per wavefront kept in registers (16 tiles per block)
  const int tile0 = blockIdx.z * 16;
  f32x4 acc[MAXT];
#pragma unroll
  for (int i = 0; i < MAXT; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
  GatherGemmArgs ga{};
  ga.mode = a.mode;
  ga.D = a.D; ga.H = a.H; ga.W = a.W;
  for (long rb = r0; rb < r1; rb += kWgRows) {
    __syncthreads();
    // stage G rows (all n) and S rows (all c) of this slab
    for (int e = threadIdx.x; e < kWgRows * a.Npad; e += 256) {
      const int rr = e / a.Npad, n = e - rr * a.Npad;
      const long r = rb + rr;
      uint16_t gv = 0;
      if (r < r1 && n < a.N) {
        long gvox = r;
        if (a.mode == GG_UP_FWD) {
          // gradient rows live at the fine voxel of tap t
          const int x = (int)(r % a.W), y = (int)((r / a.W) % a.H), z = (int)(r / ((long)a.W * a.H));
          gvox = ((long)(2 * z + (t >> 2)) * (2 * a.H) + 2 * y + ((t >> 1) & 1)) * (2 * a.W) + 2 * x + (t & 1);
        }
        gv = a.g[(size_t)gvox * a.g_cs + a.g_c0 + n];
      }
      sg[rr][n] = gv;
    }
    for (int e = threadIdx.x; e < kWgRows * a.Cpad; e += 256) {
      const int rr = e / a.Cpad, c = e - rr * a.Cpad;
      const long r = rb + rr;
      uint16_t sv = 0;
      if (r < r1 && c < a.C) {
        long svox = r;
        if (a.mode == GG_CONV3_FWD) svox = gg_source(ga, gg_row(ga, r, r + 1), t);
        if (svox >= 0) sv = a.s[(size_t)svox * a.s_cs + a.s_c0 + c];
      }
      ss[rr][c] = sv;
    }
    __syncthreads();
    // A (16 n x 32 r): lane row n = 16 tn_i + lane % 16, r = 8 (lane / 16) + 0..7
    // B (32 r x 16 c): lane column c = 16 tc_i + lane % 16
#pragma unroll
    for (int i = 0; i < MAXT; ++i) {
      const int tile = tile0 + wv + 4 * i;
      if (tile >= ntile) break;
      const int ni = tile / tc, ci = tile - ni * tc;
      uint16_t av[8], bv[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int rr = (lane >> 4) * 8 + q;
        av[q] = sg[rr][ni * 16 + (lane & 15)];
        bv[q] = ss[rr][ci * 16 + (lane & 15)];
      }
      bf16x8 A, B;
      __builtin_memcpy(&A, av, 16);
      __builtin_memcpy(&B, bv, 16);
      acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B, acc[i], 0, 0, 0);
    }
  }
  // D rows = n, columns = c
#pragma unroll
  for (int i = 0; i < MAXT; ++i) {
    const int tile = tile0 + wv + 4 * i;
    if (tile >= ntile) break;
    const int ni = tile / tc, ci = tile - ni * tc;
    const int c = ci * 16 + (lane & 15);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int n = ni * 16 + (lane >> 4) * 4 + q;
      // this block's partial (row chunk blockIdx.x); summed in chunk order by k_sum_partials
      if (n < a.N && c < a.C)
        a.part[(size_t)blockIdx.x * a.taps * a.C * a.N + ((size_t)t * a.C + c) * a.N + n] = acc[i][q];
    }
  }
}

// bias gradient: partial sums of g[r][n] over a chunk of rows per block
__global__ void __launch_bounds__(256) k_bias_grad(const uint16_t* g, int cs, int c0, int N, long nrows,
                                                   long rows_per_block, float* part) {
  const long r0 = (long)blockIdx.x * rows_per_block, r1 = min(nrows, r0 + rows_per_block);
  for (int n = threadIdx.x; n < N; n += 256) {
    float s = 0.f;
    for (long r = r0; r < r1; ++r) s += bf2f(g[(size_t)r * cs + c0 + n]);
    part[(size_t)blockIdx.x * N + n] = s;
  }
}

// out[e] += sum over b of part[b * count + e], b in order: partial sums of
// row chunks reduced the same way on every run (no floating-point atomics).
__global__ void k_sum_partials(const float* __restrict__ part, int nb, size_t count, float* out) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (size_t)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int b = 0; b < nb; ++b) s += part[(size_t)b * count + e];
    out[e] += s;
  }
}

// ---------------------------------------------------------------------------
// Max pooling 2x2x2 (forward with argmax, backward accumulating)
// ---------------------------------------------------------------------------
__global__ void k_pool_fwd(const uint16_t* x, int xcs, int xc0, uint16_t* y, int ycs, uint8_t* idx, int C,
                           int D, int H, int W) {  // D, H, W: coarse dims
  const long n = (long)D * H * W * C;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    const long q = e / C;
    const int qx = (int)(q % W), qy = (int)((q / W) % H), qz = (int)(q / ((long)W * H));
    float best = 0.f;
    int bi = 0;
    for (int d = 0; d < 8; ++d) {
      const long f = ((long)(2 * qz + (d >> 2)) * (2 * H) + 2 * qy + ((d >> 1) & 1)) * (2 * W) + 2 * qx + (d & 1);
      const float v = bf2f(x[(size_t)f * xcs + xc0 + c]);
      if (d == 0 || v > best) { best = v; bi = d; }
    }
    y[(size_t)q * ycs + c] = f2bf(best);
    idx[(size_t)q * C + c] = (uint8_t)bi;
  }
}

__global__ void k_pool_bwd(const uint16_t* gy, int gycs, const uint8_t* idx, uint16_t* gx, int gxcs, int gxc0,
                           int C, int D, int H, int W) {  // coarse dims; gx accumulates
  const long n = (long)D * H * W * C;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    const long q = e / C;
    const int qx = (int)(q % W), qy = (int)((q / W) % H), qz = (int)(q / ((long)W * H));
    const int d = idx[(size_t)q * C + c];
    const long f = ((long)(2 * qz + (d >> 2)) * (2 * H) + 2 * qy + ((d >> 1) & 1)) * (2 * W) + 2 * qx + (d & 1);
    const size_t o = (size_t)f * gxcs + gxc0 + c;
    gx[o] = f2bf(bf2f(gx[o]) + bf2f(gy[(size_t)q * gycs + c]));
  }
}

// g <- g * (y > 0) over a channel view
__global__ void k_relu_mask(uint16_t* g, int gcs, int gc0, const uint16_t* y, int ycs, int yc0, int C, long nvox) {
  const long n = nvox * C;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    const int c = (int)(e % C);
    const long v = e / C;
    if (!(bf2f(y[(size_t)v * ycs + yc0 + c]) > 0.f)) g[(size_t)v * gcs + gc0 + c] = 0;
  }
}

__global__ void k_fill_u16(uint16_t* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = 0;
}

// input: x_bf16[v][0] = scale * in[v], channels 1..cs-1 zero
__global__ void k_input(const float* in, float scale, uint16_t* x, int cs, long nvox) {
  for (long v = (long)blockIdx.x * blockDim.x + threadIdx.x; v < nvox; v += (long)gridDim.x * blockDim.x) {
    x[(size_t)v * cs] = f2bf(scale * in[v]);
    for (int c = 1; c < cs; ++c) x[(size_t)v * cs + c] = 0;
  }
}

// Weighted MSE of the head's pre-activation y (FP32) against t, weight pos_w
// where t > 0 and 1 elsewhere; gradient 2 w (y - t) / n into g[v][0]
__global__ void k_mse(const float* y, const float* t, long n, float inv_n, float pos_w, uint16_t* g, int gcs,
                      float* loss) {
  __shared__ float red[4];
  float s = 0.f;
  for (long v = (long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (long)gridDim.x * blockDim.x) {
    const float d = y[v] - t[v];
    const float w = t[v] > 0.f ? pos_w : 1.f;
    s += w * d * d;
    g[(size_t)v * gcs] = f2bf(2.f * w * d * inv_n);
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) loss[blockIdx.x] = (red[0] + red[1] + red[2] + red[3]) * inv_n;   // per-block partial
}

// Adam on FP32 master weights
// Adam.  a1 = 1 - b1, a2 = 1 - b2 and the bias corrections c1, c2 come from
// the host in FP64 (1 - 0.999f in FP32 is off by 5e-5 relative).
__global__ void k_adam(float* w, const float* g, float* m, float* v, size_t n, float lr, float b1, float b2,
                       float a1, float a2, float eps, float c1, float c2) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + a1 * gi;
    const float vi = b2 * v[i] + a2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// Pack FP32 master weights W[t][cin][cout] into BF16 B[t][n][c] for one use:
// transpose = 1: n = cout, c = cin (forward); 0: n = cin, c = cout (input
// gradient).  Channels beyond the real counts are zero.
__global__ void k_pack(const float* w, int T, int cin, int cout, int transpose, int Npad, int Cpad, uint16_t* out) {
  const size_t n = (size_t)T * Npad * Cpad;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % Cpad);
    const int nn = (int)((e / Cpad) % Npad);
    const int t = (int)(e / ((size_t)Cpad * Npad));
    float v = 0.f;
    if (transpose) {
      if (nn < cout && c < cin) v = w[((size_t)t * cin + c) * cout + nn];
    } else {
      if (nn < cin && c < cout) v = w[((size_t)t * cin + nn) * cout + c];
    }
    out[e] = f2bf(v);
  }
}

// Up-convolution forward packing: B[0][n = d*cout + co][c = ci] = U[d][ci][co].
__global__ void k_pack_up_fwd(const float* u, int cin, int cout, uint16_t* out) {
  const size_t n = (size_t)8 * cout * cin;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
    const int ci = (int)(e % cin);
    const int col = (int)(e / cin);
    const int d = col / cout, co = col - d * cout;
    out[e] = f2bf(u[((size_t)d * cin + ci) * cout + co]);
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
__global__ void k_fill_f32_one(float* p) {
  if (threadIdx.x == 0) *p = 0.f;
}

static int ew_grid(size_t n) {
  size_t b = (n + 255) / 256;
  return (int)(b > 16384 ? 16384 : (b == 0 ? 1 : b));
}

// Halo-box bytes of k_conv3_lds, or 0 when a layer does not take it (other
// modes, more than 8 column tiles, rows narrower than a tile, or a box above
// 64 KiB, which would leave fewer than two blocks per CU).
static size_t conv3_lds_bytes(const GatherGemmArgs& a, int rt) {
  if (a.mode != GG_CONV3_FWD && a.mode != GG_CONV3_BWD) return 0;
  if (a.Npad / 16 > 8 || a.W < 16 || a.C % 8 != 0 || a.src_cs % 8 != 0 || a.src_c0 % 8 != 0) return 0;
  const size_t bytes = (size_t)kHbX * kHbY * (rt + 2) * a.C * sizeof(uint16_t);
  return bytes <= 64 * 1024 ? bytes : 0;
}

hipError_t launch_gather_gemm(const GatherGemmArgs& a, hipStream_t s) {
  const long nrows = (long)a.D * a.H * a.W;
  {
    const int nb = a.Npad / 16;
    const int rt = nb <= 2 ? 4 : (nb == 4 ? 2 : 1);
    const size_t lds = conv3_lds_bytes(a, rt);
    if (lds > 0) {
      const dim3 g((unsigned)((a.W + 15) / 16), (unsigned)((a.H + 3) / 4), (unsigned)((a.D + rt - 1) / rt));
      const bool bwd = a.mode == GG_CONV3_BWD;
#define RIHVR_CONV3(NB, RT)                                                                                    \
  if (bwd) hipLaunchKernelGGL((k_conv3_lds<NB, RT, GG_CONV3_BWD>), g, dim3(256), lds, s, a);                   \
  else hipLaunchKernelGGL((k_conv3_lds<NB, RT, GG_CONV3_FWD>), g, dim3(256), lds, s, a);
      switch (nb) {
        case 1: RIHVR_CONV3(1, 4) break;
        case 2: RIHVR_CONV3(2, 4) break;
        case 4: RIHVR_CONV3(4, 2) break;
        case 8: RIHVR_CONV3(8, 1) break;
        default: return hipErrorInvalidValue;
      }
#undef RIHVR_CONV3
      return hipGetLastError();
    }
  }
  // row tiles per wave: enough MFMAs per loaded fragment without exceeding the
  // accumulator budget (RT * NB <= 8 tiles of 16 x 16)
  auto grid = [&](int rt) { return dim3((unsigned)((nrows + 64 * rt - 1) / (64 * rt))); };
  auto by_mode = [&](auto nb, auto rt) -> hipError_t {
    constexpr int NB = decltype(nb)::value, RT = decltype(rt)::value;
    const dim3 g = grid(RT);
    switch (a.mode) {
      case GG_CONV3_FWD: hipLaunchKernelGGL((k_gather_gemm<NB, RT, GG_CONV3_FWD>), g, dim3(256), 0, s, a); break;
      case GG_CONV3_BWD: hipLaunchKernelGGL((k_gather_gemm<NB, RT, GG_CONV3_BWD>), g, dim3(256), 0, s, a); break;
      case GG_UP_BWD: hipLaunchKernelGGL((k_gather_gemm<NB, RT, GG_UP_BWD>), g, dim3(256), 0, s, a); break;
      case GG_UP_FWD:
      case GG_POINT: hipLaunchKernelGGL((k_gather_gemm<NB, RT, GG_POINT>), g, dim3(256), 0, s, a); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  };
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  using I4 = std::integral_constant<int, 4>;
  switch (a.Npad / 16) {
    case 1: return by_mode(I1{}, I4{});
    case 2: return by_mode(I2{}, I4{});
    case 4: return by_mode(I4{}, I2{});
    case 8: return by_mode(std::integral_constant<int, 8>{}, I1{});
    case 16: return by_mode(std::integral_constant<int, 16>{}, I1{});
    case 32: return by_mode(std::integral_constant<int, 32>{}, I1{});
    case 64: return by_mode(std::integral_constant<int, 64>{}, I1{});
    default: return hipErrorInvalidValue;
  }
}

long wgrad_rows_per_block(long nrows) { return std::max<long>(2048, (nrows + kReduceBlocks - 1) / kReduceBlocks); }
long bias_rows_per_block(long nrows) { return std::max<long>(4096, (nrows + kReduceBlocks - 1) / kReduceBlocks); }

hipError_t launch_wgrad(WgradArgs a, int taps, float* part, hipStream_t s) {
  if (a.Npad > kWgMaxN || a.Cpad > kWgMaxC || a.Npad % 16 || a.Cpad % 16) return hipErrorInvalidValue;
  const long nrows = (long)a.D * a.H * a.W;
  a.rows_per_block = wgrad_rows_per_block(nrows);
  a.taps = taps;
  a.part = part;
  const int nb = (int)((nrows + a.rows_per_block - 1) / a.rows_per_block);
  const int groups = ((a.Npad / 16) * (a.Cpad / 16) + 15) / 16;
  hipLaunchKernelGGL(k_wgrad, dim3(nb, taps, groups), dim3(256), 0, s, a);
  const size_t count = (size_t)taps * a.C * a.N;
  hipLaunchKernelGGL(k_sum_partials, dim3(ew_grid(count)), dim3(256), 0, s, part, nb, count, a.dw);
  return hipGetLastError();
}

hipError_t launch_bias_grad(const uint16_t* g, int cs, int c0, int N, long nrows, float* db, float* part,
                            hipStream_t s) {
  const long per = bias_rows_per_block(nrows);
  const int nb = (int)((nrows + per - 1) / per);
  hipLaunchKernelGGL(k_bias_grad, dim3(nb), dim3(256), 0, s, g, cs, c0, N, nrows, per, part);
  hipLaunchKernelGGL(k_sum_partials, dim3(ew_grid((size_t)N)), dim3(256), 0, s, part, nb, (size_t)N, db);
  return hipGetLastError();
}

hipError_t launch_pool_fwd(const uint16_t* x, int xcs, int xc0, uint16_t* y, int ycs, uint8_t* idx, int C, int D,
                           int H, int W, hipStream_t s) {
  hipLaunchKernelGGL(k_pool_fwd, dim3(ew_grid((size_t)D * H * W * C)), dim3(256), 0, s, x, xcs, xc0, y, ycs, idx, C,
                     D, H, W);
  return hipGetLastError();
}

hipError_t launch_pool_bwd(const uint16_t* gy, int gycs, const uint8_t* idx, uint16_t* gx, int gxcs, int gxc0, int C,
                           int D, int H, int W, hipStream_t s) {
  hipLaunchKernelGGL(k_pool_bwd, dim3(ew_grid((size_t)D * H * W * C)), dim3(256), 0, s, gy, gycs, idx, gx, gxcs,
                     gxc0, C, D, H, W);
  return hipGetLastError();
}

hipError_t launch_relu_mask(uint16_t* g, int gcs, int gc0, const uint16_t* y, int ycs, int yc0, int C, long nvox,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_relu_mask, dim3(ew_grid((size_t)nvox * C)), dim3(256), 0, s, g, gcs, gc0, y, ycs, yc0, C,
                     nvox);
  return hipGetLastError();
}

hipError_t launch_zero_u16(uint16_t* p, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u16, dim3(ew_grid(n)), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_input(const float* in, float scale, uint16_t* x, int cs, long nvox, hipStream_t s) {
  hipLaunchKernelGGL(k_input, dim3(ew_grid(nvox)), dim3(256), 0, s, in, scale, x, cs, nvox);
  return hipGetLastError();
}

hipError_t launch_mse(const float* y, const float* t, long n, float pos_w, uint16_t* g, int gcs, float* loss,
                      float* part, hipStream_t s) {
  // per-block partials in part (ew_grid(n) <= kLossBlocks of them), then one ordered sum
  const int nb = ew_grid(n);
  hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, s, y, t, n, 1.f / (float)n, pos_w, g, gcs, part);
  hipLaunchKernelGGL(k_fill_f32_one, dim3(1), dim3(64), 0, s, loss);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, part, nb, (size_t)1, loss);
  return hipGetLastError();
}

hipError_t launch_adam(float* w, const float* g, float* m, float* v, size_t n, float lr, double b1, double b2,
                       double eps, int step, hipStream_t s) {
  const float c1 = (float)(1.0 - std::pow(b1, (double)step)), c2 = (float)(1.0 - std::pow(b2, (double)step));
  hipLaunchKernelGGL(k_adam, dim3(ew_grid(n)), dim3(256), 0, s, w, g, m, v, n, lr, (float)b1, (float)b2,
                     (float)(1.0 - b1), (float)(1.0 - b2), (float)eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_pack(const float* w, int T, int cin, int cout, int transpose, int Npad, int Cpad, uint16_t* out,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_pack, dim3(ew_grid((size_t)T * Npad * Cpad)), dim3(256), 0, s, w, T, cin, cout, transpose,
                     Npad, Cpad, out);
  return hipGetLastError();
}

hipError_t launch_pack_up_fwd(const float* u, int cin, int cout, uint16_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_up_fwd, dim3(ew_grid((size_t)8 * cin * cout)), dim3(256), 0, s, u, cin, cout, out);
  return hipGetLastError();
}

}  // namespace rihvr
