// HIP kernels for gfx950: the forward model A, its adjoint fused with the
// FISTA gradient step, the hologram-space residual, objective partials and the
// on-device FISTA scalars.
//
// Spectra use the packed real-to-complex layout: a real row of nx samples is
// transformed as nx/2 complex samples z[n] = x[2n] + i x[2n+1], and its
// spectrum is stored as m = nx/2 complex values with slot 0 holding
// X[0] + i X[nx/2] (both real) and slots 1..m-1 holding X[1..m-1].  In 2D the
// packed column 0 then carries the DC and Nyquist columns as one complex
// column (each of them is the spectrum of a real sequence), so a plane's
// half spectrum is exactly ny x m complex values, the same bytes as the real
// plane.
//
// Because the fftfreq grid is symmetric and H_j(f) = H_j(-f), for real x
// Re(IFFT2(FFT2(x) H_j)) = IFFT2(FFT2(x) cos(phi_j)), phi_j = arg H_j, so both A
// and A^T apply the real, even filter cos(phi_j) to half spectra.  For the packed
// column 0 the DC and Nyquist columns get different filters c0, cN; with
// Z = FFT(dc) + i FFT(nyq), the filtered packed column is
// ((c0 + cN)/2) Z[ky] + ((c0 - cN)/2) conj(Z[-ky]).
//
// The phase phi_j(f) = 2 pi (c_j + z_j theta(f)), theta(f) = sqrt(1/lambda^2 -
// f^2) - 1/lambda, c_j = frac(z_j / lambda), reaches ~10^2 cycles, so it is
// reduced modulo one cycle in FP64 before an FP32 cospi.
#include "rihvr_internal.h"
#include "fft_device.h"

namespace rihvr {

// ---------------------------------------------------------------------------
// Launch-shape choices
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int kRowThreads(int m) { return m / points_per_thread(m); }
__host__ __device__ constexpr int kRowsPerBlock(int m) {
  return kRowThreads(m) >= 256 ? 1 : 256 / kRowThreads(m);
}
// Row transforms of at most 64 threads lie inside one wavefront each: their
// passes order LDS within the wave, with no block barrier.
__host__ __device__ constexpr bool kRowWave(int m) { return kRowThreads(m) <= 64; }
// Column transforms: points per thread, and columns per tile such that a block
// has at most 512 threads (256 VGPRs per lane available, no spills) and the tile
// plus three column-sized tables (a column buffer, the twiddles, the Nyquist
// column's theta) and 4 KiB of flags fit the 160 KiB of LDS.
__host__ __device__ constexpr int kColP(int ny) { return (ny % 3 == 0) ? 12 : (ny >= 2048 ? 16 : 8); }
__host__ __device__ constexpr int kColW(int ny) {
  int w = 16;
  while (w > 1 && ((ny / kColP(ny)) * w > 512 || (size_t)ny * (w + 3) * 8 + 4096 > 160 * 1024)) w /= 2;
  return w;
}

int rows_per_block(int m) { return kRowsPerBlock(m); }
int col_tile_width(int ny) { return kColW(ny); }
bool fft_len_supported(int L) {
  switch (L) {
    case 8: case 16: case 32: case 64: case 128: case 256: case 512: case 1024: case 2048:
    case 24: case 48: case 96: case 192: case 384: case 768: case 1536:
      return true;
    default: return false;
  }
}

__device__ __forceinline__ float phase_cos(double z, double c, double th) {
  double ph = fma(z, th, c);
  ph -= floor(ph);
  return cospif(2.0f * (float)ph);
}

__device__ __forceinline__ bool solve_done(const SolveState* st) {
  return st != nullptr && st->done != 0;
}

// Block-wide FP64 sum; result valid in thread 0.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  constexpr int NW = (NT + 63) / 64;
  if constexpr (NW > 1) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) red[wid] = v;
    __syncthreads();
    v = 0.0;
    if (threadIdx.x < NW) v = red[threadIdx.x];
    if (wid == 0) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    }
  }
  return v;
}

// ---------------------------------------------------------------------------
// Packed R2C of real rows.  Block: ROWS rows x T threads; each row in LDS.
// ---------------------------------------------------------------------------
template <int M>
__device__ __forceinline__ void rows_r2c_body(const RowsR2CArgs& a, int bx, int by) {
  const float2* __restrict__ tw = a.pt.tw_row;
  constexpr int P = points_per_thread(M), T = M / P, ROWS = kRowsPerBlock(M);
  __shared__ float2 lds[ROWS][M];
  if (solve_done(a.st)) return;
  constexpr bool WAVE = kRowWave(M);
  const int r = threadIdx.x / T, t = threadIdx.x % T;
  const int row = bx * ROWS + r;
  const bool active = row < a.nrows && (a.rowflag == nullptr || a.rowflag[row] != 0);
  if constexpr (WAVE) {
    if (__ballot(active) == 0) return;   // no row of this wave is occupied
  } else {
    if (!__syncthreads_or(active)) return;
  }
  float2* buf = lds[r];
  if (a.mode != 1) {
    const float2* src = nullptr;
    if (a.mode == 2 && a.rs.on) {
      // solver iterate from its row store (an absent row is all zero)
      if (row < a.nrows) src = reinterpret_cast<const float2*>(store_row(a.rs, a.st->it & 1, (size_t)row));
    } else {
      const float* xin = a.x;
      if (a.mode == 2) xin = pick3(a.xs[0], a.xs[1], a.xs[2], a.st->it % 3);   // solver iterate, before the scalar kernel
      src = reinterpret_cast<const float2*>(xin) + (size_t)row * M;
    }
#pragma unroll
    for (int s = 0; s < P; ++s) {
      const int e = t + s * T;
      buf[e] = (active && src != nullptr) ? src[e] : make_float2(0.f, 0.f);
    }
  } else {
    const SolveState* st = a.st;
    const float beta = (float)st->beta;
    const float2* c0 = reinterpret_cast<const float2*>(st->ax_cur ? a.ax1 : a.ax0) + (size_t)row * M;
    const float2* c1 = reinterpret_cast<const float2*>(st->ax_prev ? a.ax1 : a.ax0) + (size_t)row * M;
    const float2* bb = reinterpret_cast<const float2*>(a.b) + (size_t)row * M;
#pragma unroll
    for (int s = 0; s < P; ++s) {
      const int e = t + s * T;
      float2 v = make_float2(0.f, 0.f);
      if (active) {
        float2 xc = c0[e], xp = c1[e], bv = bb[e];
        v.x = xc.x + beta * (xc.x - xp.x) - bv.x;
        v.y = xc.y + beta * (xc.y - xp.y) - bv.y;
      }
      buf[e] = v;
    }
  }
  lds_sync<WAVE>();
  fft_lds<M, P, 1, 2, false, WAVE>(buf, t, tw);
  if (!active) return;  // no barriers below
  float2* dst = a.out + (size_t)row * M;
#pragma unroll
  for (int s = 0; s < P; ++s) {
    const int k = t + s * T;
    const float2 zk = buf[k];
    float2 o;
    if (k == 0) {
      o = make_float2(zk.x + zk.y, zk.x - zk.y);
    } else {
      const float2 zm = cconj(buf[M - k]);
      const float2 e = cscale(cadd(zk, zm), 0.5f);
      const float2 d = csub(zk, zm);
      const float2 od = make_float2(0.5f * d.y, -0.5f * d.x);  // (zk - zm) / (2i)
      o = cadd(e, cmul(tw[k], od));
    }
    dst[k] = o;
  }
}

// ---------------------------------------------------------------------------
// Packed C2R of rows (scaled).  Inverse of k_rows_r2c up to the scale.
// ---------------------------------------------------------------------------
template <int M, bool WAVE>
__device__ __forceinline__ void c2r_prepare(float2* buf, int t, const float2* __restrict__ tw) {
  constexpr int P = points_per_thread(M), T = M / P;
  float2 zt[P];
#pragma unroll
  for (int s = 0; s < P; ++s) {
    const int k = t + s * T;
    const float2 xk = buf[k];
    if (k == 0) {
      zt[s] = make_float2(xk.x + xk.y, xk.x - xk.y);
    } else {
      const float2 xc = cconj(buf[M - k]);
      const float2 sum = cadd(xk, xc), dif = csub(xk, xc);
      const float2 wd = cmulc(dif, tw[k]);             // exp(+2 pi i k / nx) * dif
      zt[s] = make_float2(sum.x - wd.y, sum.y + wd.x);  // sum + i wd
    }
  }
  lds_sync<WAVE>();
#pragma unroll
  for (int s = 0; s < P; ++s) buf[t + s * T] = zt[s];
  lds_sync<WAVE>();
}

template <int M>
__device__ __forceinline__ void rows_c2r_body(const RowsC2RArgs& a, int bx, int by) {
  const float2* __restrict__ tw = a.pt.tw_row;
  constexpr int P = points_per_thread(M), T = M / P, ROWS = kRowsPerBlock(M), NT = ROWS * T;
  __shared__ float2 lds[ROWS][M];
  __shared__ double red[16];
  if (solve_done(a.st)) return;
  const int r = threadIdx.x / T, t = threadIdx.x % T;
  const int row = bx * ROWS + r;
  const bool active = row < a.nrows;
  float2* buf = lds[r];
  const float2* src = a.in + (size_t)row * M;
#pragma unroll
  for (int s = 0; s < P; ++s) {
    const int e = t + s * T;
    buf[e] = active ? src[e] : make_float2(0.f, 0.f);
  }
  lds_sync<kRowWave(M)>();
  c2r_prepare<M, kRowWave(M)>(buf, t, tw);
  fft_lds<M, P, 1, 2, true, kRowWave(M)>(buf, t, tw);
  if (a.mode == 0) {
    if (!active) return;
    float2* dst = reinterpret_cast<float2*>(a.out) + (size_t)row * M;
#pragma unroll
    for (int s = 0; s < P; ++s) dst[t + s * T] = cscale(buf[t + s * T], a.scale);
    return;
  }
  double acc = 0.0;
  if (active) {
    // runs before the scalar kernel of the iteration: A x_it goes to slot it & 1
    float2* dst = reinterpret_cast<float2*>((a.st->it & 1) ? a.ax1 : a.ax0) + (size_t)row * M;
    const float2* bb = reinterpret_cast<const float2*>(a.b) + (size_t)row * M;
#pragma unroll
    for (int s = 0; s < P; ++s) {
      const int e = t + s * T;
      const float2 v = cscale(buf[e], a.scale);
      dst[e] = v;
      const float2 bv = bb[e];
      const double dx = (double)v.x - (double)bv.x, dy = (double)v.y - (double)bv.y;
      acc += dx * dx + dy * dy;
    }
  }
  acc = block_sum<NT>(acc, red);
  if (threadIdx.x == 0) a.partial[bx] = 0.5 * acc;
}

// ---------------------------------------------------------------------------
// Column-kernel helpers.  The column transforms run once per plane with the
// same twiddles, so each block copies the table into LDS once: read from
// global memory inside the passes, every twiddle load also waits for the
// prefetched tile of the next plane (vector loads complete in order).  For the
// same reason the tile loads are branch-free buffer loads: a load whose lane
// is switched off by a row flag takes an offset past the end of the plane's
// buffer descriptor and returns zero.
// ---------------------------------------------------------------------------
constexpr unsigned kColOff = 0x80000000u;   // past every plane descriptor: reads 0
constexpr int kColPlaneFlags = 2048;        // plane flags of a chunk staged in LDS

__device__ __forceinline__ __amdgpu_buffer_rsrc_t spec_rsrc(const float2* plane, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float2*>(plane), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float2 buf_ld2(__amdgpu_buffer_rsrc_t r, unsigned off) {
  const auto u = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0);
  return make_float2(__uint_as_float(u[0]), __uint_as_float(u[1]));
}
template <int NY>
__device__ __forceinline__ void stage_twiddles(float2* s_tw, const float2* __restrict__ tw) {
  for (int i = threadIdx.x; i < NY; i += blockDim.x) s_tw[i] = tw[i];
}
// theta of the Nyquist column (kx = m), which column 0 pairs with; only the
// block holding column 0 needs it.
template <int NY>
__device__ __forceinline__ void stage_theta_nyquist(double* s_thn, const double* __restrict__ theta, int m,
                                                    bool needed) {
  if (needed)
    for (int i = threadIdx.x; i < NY; i += blockDim.x) s_thn[i] = theta[(size_t)i * (m + 1) + m];
}

// ---------------------------------------------------------------------------
// Forward column pass with the propagation filter and the sum over planes.
// Block: W columns x TC threads per column (TC = NY / P).
// ---------------------------------------------------------------------------
//
// Software pipeline over the planes of the chunk: the tile of the next
// non-empty plane is requested right after the barrier that precedes the
// transform of the current one, so its loads run under the transform; the row
// flags that decide which rows of that tile are read are themselves staged
// into LDS one plane earlier still (one dword of flags per thread).
// Direct form (no prefetch) for the transform sizes whose pipelined form would
// not fit the register file: every row flag is read from global memory.
template <int NY>
__device__ __forceinline__ void fwd_cols_body_direct(const FwdColsArgs& a, int bx, int by) {
  const PlanTables& pt = a.pt;
  constexpr int P = kColP(NY), TC = NY / P, W = kColW(NY);
  __shared__ float2 lds[NY * W];
  __shared__ float2 s_tw[NY];
  __shared__ double s_thn[NY];
  if (solve_done(a.st)) return;
  const int w = threadIdx.x % W, q = threadIdx.x / W;
  const int m = a.m;
  const int kx = bx * W + w;
  const bool colok = kx < m;           // tiles may overhang the last column
  const bool col0 = (kx == 0);
  // first read after the loop's first barrier
  stage_twiddles<NY>(s_tw, pt.tw_col);
  stage_theta_nyquist<NY>(s_thn, pt.theta, m, bx == 0);
  double th[P];
#pragma unroll
  for (int s = 0; s < P; ++s) th[s] = colok ? pt.theta[(size_t)(q + s * TC) * (m + 1) + kx] : 0.0;
  float2 acc[P];
#pragma unroll
  for (int s = 0; s < P; ++s) acc[s] = make_float2(0.f, 0.f);
  const int j0 = by * a.planes_per_chunk;
  const int j1 = min(a.nz, j0 + a.planes_per_chunk);
  for (int j = j0; j < j1; ++j) {
    if (a.planeflag != nullptr && a.planeflag[j] == 0) continue;
    const float2* src = a.t + (size_t)j * NY * m + kx;
#pragma unroll
    for (int s = 0; s < P; ++s) {
      const int y = q + s * TC;
      const bool on = colok && (a.rowflag == nullptr || a.rowflag[(size_t)j * NY + y] != 0);
      lds[y * W + w] = on ? src[(size_t)y * m] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    fft_lds<NY, P, W, 1, false>(lds + w, q, s_tw);
    const double2 zc = pt.zc[j];
#pragma unroll
    for (int s = 0; s < P; ++s) {
      const int y = q + s * TC;
      const float2 v = lds[y * W + w];
      const float c = phase_cos(zc.x, zc.y, th[s]);
      if (!col0) {
        acc[s].x += c * v.x;
        acc[s].y += c * v.y;
      } else {
        const float cn = phase_cos(zc.x, zc.y, s_thn[y]);
        const float2 vn = cconj(lds[((NY - y) % NY) * W]);
        const float ca = 0.5f * (c + cn), cb = 0.5f * (c - cn);
        acc[s].x += ca * v.x + cb * vn.x;
        acc[s].y += ca * v.y + cb * vn.y;
      }
    }
    __syncthreads();
  }
  if (!colok) return;
  float2* dst = a.gp + (size_t)by * NY * m + kx;
#pragma unroll
  for (int s = 0; s < P; ++s) dst[(size_t)(q + s * TC) * m] = acc[s];
}

template <int NY>
__device__ __forceinline__ void fwd_cols_body(const FwdColsArgs& a, int bx, int by) {
  if constexpr (kColP(NY) > 8) {
    fwd_cols_body_direct<NY>(a, bx, by);
    return;
  }
  const PlanTables& pt = a.pt;
  constexpr int P = kColP(NY), TC = NY / P, W = kColW(NY);
  constexpr int NFW = NY / 4;          // dwords of row flags per plane
  static_assert(W * TC >= NFW, "one flag dword per thread");
  __shared__ float2 lds[NY * W];
  __shared__ uint32_t lds_fl[NFW];
  __shared__ float2 s_tw[NY];
  __shared__ double s_thn[NY];
  __shared__ uint8_t s_pf[kColPlaneFlags];
  if (solve_done(a.st)) return;
  const int w = threadIdx.x % W, q = threadIdx.x / W;
  const int m = a.m;
  const int kx = bx * W + w;
  const bool colok = kx < m;           // tiles may overhang the last column
  const bool col0 = (kx == 0);
  const bool flags = a.rowflag != nullptr;
  const uint8_t* fl8 = reinterpret_cast<const uint8_t*>(lds_fl);
  double th[P];
#pragma unroll
  for (int s = 0; s < P; ++s) th[s] = colok ? pt.theta[(size_t)(q + s * TC) * (m + 1) + kx] : 0.0;
  float2 acc[P];
#pragma unroll
  for (int s = 0; s < P; ++s) acc[s] = make_float2(0.f, 0.f);
  const int j0 = by * a.planes_per_chunk;
  const int j1 = min(a.nz, j0 + a.planes_per_chunk);
  // the chunk's plane flags (planes past the staged range count as occupied)
  const bool pflags = a.planeflag != nullptr;
  if (pflags)
    for (int i = threadIdx.x; i < min(j1 - j0, kColPlaneFlags); i += blockDim.x) s_pf[i] = a.planeflag[j0 + i];
  stage_twiddles<NY>(s_tw, pt.tw_col);
  stage_theta_nyquist<NY>(s_thn, pt.theta, m, bx == 0);
  __syncthreads();
  auto next_plane = [&](int j) {
    if (pflags)
      while (j < j1 && j - j0 < kColPlaneFlags && s_pf[j - j0] == 0) ++j;
    return j;
  };
  auto load_flagword = [&](int j) -> uint32_t {
    return reinterpret_cast<const uint32_t*>(a.rowflag + (size_t)j * NY)[threadIdx.x];
  };
  float2 nv[P];  // tile of the next plane, in flight
  const size_t plane_bytes = (size_t)NY * m * sizeof(float2);
  auto load_tile = [&](int j) {
    const __amdgpu_buffer_rsrc_t r = spec_rsrc(a.t + (size_t)j * NY * m, plane_bytes);
    // offsets first (the flag bytes are read even when unused), then the loads
    unsigned o[P];
#pragma unroll
    for (int s = 0; s < P; ++s) {
      const int y = q + s * TC;
      const bool on = colok & (!flags | (fl8[y] != 0));
      o[s] = on ? (unsigned)((y * m + kx) * sizeof(float2)) : kColOff;
    }
#pragma unroll
    for (int s = 0; s < P; ++s) nv[s] = buf_ld2(r, o[s]);
  };
  int j = next_plane(j0);
  int jn = j < j1 ? next_plane(j + 1) : j1;
  uint32_t flw = 0;  // flag dword of plane jn (threads < NFW)
  if (j < j1) {
    if (flags) {
      if (threadIdx.x < NFW) lds_fl[threadIdx.x] = load_flagword(j);
      __syncthreads();
    }
    load_tile(j);
    if (flags && jn < j1 && threadIdx.x < NFW) flw = load_flagword(jn);
    __syncthreads();  // the flags of j are read before the loop overwrites them
  }
  while (j < j1) {
#pragma unroll
    for (int s = 0; s < P; ++s) lds[(q + s * TC) * W + w] = nv[s];
    if (flags && jn < j1 && threadIdx.x < NFW) lds_fl[threadIdx.x] = flw;
    const int jnn = jn < j1 ? next_plane(jn + 1) : j1;
    if (flags && jnn < j1 && threadIdx.x < NFW) flw = load_flagword(jnn);
    __syncthreads();
    if (jn < j1) load_tile(jn);
    fft_lds<NY, P, W, 1, false>(lds + w, q, s_tw);
    const double2 zc = pt.zc[j];
#pragma unroll
    for (int s = 0; s < P; ++s) {
      const int y = q + s * TC;
      const float2 v = lds[y * W + w];
      const float c = phase_cos(zc.x, zc.y, th[s]);
      if (!col0) {
        acc[s].x += c * v.x;
        acc[s].y += c * v.y;
      } else {
        const float cn = phase_cos(zc.x, zc.y, s_thn[y]);
        const float2 vn = cconj(lds[((NY - y) % NY) * W]);
        const float ca = 0.5f * (c + cn), cb = 0.5f * (c - cn);
        acc[s].x += ca * v.x + cb * vn.x;
        acc[s].y += ca * v.y + cb * vn.y;
      }
    }
    __syncthreads();
    j = jn;
    jn = jnn;
  }
  if (!colok) return;
  float2* dst = a.gp + (size_t)by * NY * m + kx;
#pragma unroll
  for (int s = 0; s < P; ++s) dst[(size_t)(q + s * TC) * m] = acc[s];
}

// ---------------------------------------------------------------------------
// Sum of partial spectra and inverse column FFT (hologram sized).
// ---------------------------------------------------------------------------
template <int NY>
__device__ __forceinline__ void holo_cols_inv_body(const HoloColsInvArgs& a, int bx, int by) {
  const PlanTables& pt = a.pt;
  constexpr int P = kColP(NY), TC = NY / P, W = kColW(NY);
  __shared__ float2 lds[NY * W];
  if (solve_done(a.st)) return;
  const int w = threadIdx.x % W, q = threadIdx.x / W;
  const int m = a.m;
  const int kx = bx * W + w;
#pragma unroll
  for (int s = 0; s < P; ++s) {
    const int y = q + s * TC;
    float2 v = make_float2(0.f, 0.f);
    if (kx < m)
      for (int c = 0; c < a.nchunk; ++c) v = cadd(v, a.gp[((size_t)c * NY + y) * m + kx]);
    lds[y * W + w] = v;
  }
  __syncthreads();
  fft_lds<NY, P, W, 1, true>(lds + w, q, pt.tw_col);
  if (kx >= m) return;
#pragma unroll
  for (int s = 0; s < P; ++s) {
    const int y = q + s * TC;
    a.gi[(size_t)y * m + kx] = lds[y * W + w];
  }
}

// ---------------------------------------------------------------------------
// Adjoint column pass.  The residual spectrum of the tile is computed once
// (column FFT of its packed row spectra) and kept in registers; every plane of
// the chunk multiplies it by cos(phase_j) and inverse-transforms the columns.
// ---------------------------------------------------------------------------
template <int NY>
__device__ __forceinline__ void adj_cols_body(const AdjColsArgs& a, int bx, int by) {
  const PlanTables& pt = a.pt;
  constexpr int P = kColP(NY), TC = NY / P, W = kColW(NY);
  __shared__ float2 lds[NY * W];
  __shared__ float2 r0[NY];
  __shared__ float2 s_tw[NY];
  __shared__ double s_thn[NY];
  if (solve_done(a.st)) return;
  const int w = threadIdx.x % W, q = threadIdx.x / W;
  const int m = a.m;
  const int kx = bx * W + w;
  const bool colok = kx < m;
  const bool col0 = (kx == 0);
  stage_twiddles<NY>(s_tw, pt.tw_col);
  stage_theta_nyquist<NY>(s_thn, pt.theta, m, bx == 0);
#pragma unroll
  for (int s = 0; s < P; ++s) {
    const int y = q + s * TC;
    lds[y * W + w] = colok ? a.th[(size_t)y * m + kx] : make_float2(0.f, 0.f);
  }
  __syncthreads();
  fft_lds<NY, P, W, 1, false>(lds + w, q, s_tw);
  float2 rh[P];
  double th[P];
#pragma unroll
  for (int s = 0; s < P; ++s) {
    const int y = q + s * TC;
    rh[s] = lds[y * W + w];
    if (w == 0) r0[y] = rh[s];
    th[s] = colok ? pt.theta[(size_t)y * (m + 1) + kx] : 0.0;
  }
  __syncthreads();
  const int j0 = by * a.planes_per_chunk;
  const int j1 = min(a.nz, j0 + a.planes_per_chunk);
  for (int j = j0; j < j1; ++j) {
    const double2 zc = pt.zc[j];
#pragma unroll
    for (int s = 0; s < P; ++s) {
      const int y = q + s * TC;
      const float c = phase_cos(zc.x, zc.y, th[s]);
      float2 v;
      if (!col0) {
        v = cscale(rh[s], c);
      } else {
        const float cn = phase_cos(zc.x, zc.y, s_thn[y]);
        const float2 vn = cconj(r0[(NY - y) % NY]);
        const float ca = 0.5f * (c + cn), cb = 0.5f * (c - cn);
        v = make_float2(ca * rh[s].x + cb * vn.x, ca * rh[s].y + cb * vn.y);
      }
      lds[y * W + w] = v;
    }
    __syncthreads();
    fft_lds<NY, P, W, 1, true>(lds + w, q, s_tw);
    float2* dst = a.u + (size_t)j * NY * m + kx;
    if (colok) {
#pragma unroll
      for (int s = 0; s < P; ++s) {
        const int y = q + s * TC;
        dst[(size_t)y * m] = lds[y * W + w];
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Adjoint row pass: packed C2R, then either store A^T r or the gradient step
// v = y - t A^T r with the extrapolated point y formed on the fly.
// ---------------------------------------------------------------------------
template <int M>
__device__ __forceinline__ void adj_rows_body(const AdjRowsArgs& a, int bx, int by) {
  const float2* __restrict__ tw = a.pt.tw_row;
  constexpr int P = points_per_thread(M), T = M / P, ROWS = kRowsPerBlock(M);
  __shared__ float2 lds[ROWS][M];
  if (solve_done(a.st)) return;
  const int r = threadIdx.x / T, t = threadIdx.x % T;
  const int row = bx * ROWS + r;
  const bool active = row < a.nrows;
  // gradient step: a row of x_k or x_{k-1} whose flag is clear is all zero and
  // is not read (flags read here, before the row's transform; cleared below)
  bool fc = true, fp = true;
  if (a.mode == 1 && a.rowflag_prev != nullptr && active) {
    fc = a.rowflag[row] != 0;
    fp = a.rowflag_prev[row] != 0;
  }
  float2* buf = lds[r];
  const float2* src = a.u + (size_t)row * M;
#pragma unroll
  for (int s = 0; s < P; ++s) {
    const int e = t + s * T;
    buf[e] = active ? src[e] : make_float2(0.f, 0.f);
  }
  lds_sync<kRowWave(M)>();
  c2r_prepare<M, kRowWave(M)>(buf, t, tw);
  fft_lds<M, P, 1, 2, true, kRowWave(M)>(buf, t, tw);
  if (!active) return;
  if (a.mode == 0) {
    float2* dst = reinterpret_cast<float2*>(a.out) + (size_t)row * M;
#pragma unroll
    for (int s = 0; s < P; ++s) dst[t + s * T] = cscale(buf[t + s * T], a.scale);
    return;
  }
  const SolveState* st = a.st;
  const float2* xc;
  const float2* xpr;
  float2* vo;
  if (a.rs.on) {
    // iterates from their row stores; v into the dense prox input
    xc = fc ? reinterpret_cast<const float2*>(store_row(a.rs, st->scur, (size_t)row)) : nullptr;
    xpr = fp ? reinterpret_cast<const float2*>(store_row(a.rs, st->scur ^ 1, (size_t)row)) : nullptr;
    vo = reinterpret_cast<float2*>(a.rs.v) + (size_t)row * M;
  } else {
    xc = fc ? reinterpret_cast<const float2*>(pick3(a.x0, a.x1, a.x2, st->cur)) + (size_t)row * M : nullptr;
    vo = reinterpret_cast<float2*>(pick3(a.x0, a.x1, a.x2, st->prev)) + (size_t)row * M;
    xpr = fp ? vo : nullptr;
  }
  const float beta = (float)st->beta;
  const float gs = (float)(a.step * (double)a.scale);
#pragma unroll
  for (int s = 0; s < P; ++s) {
    const int e = t + s * T;
    const float2 g = buf[e];
    const float2 c = xc != nullptr ? xc[e] : make_float2(0.f, 0.f);
    const float2 p = xpr != nullptr ? xpr[e] : make_float2(0.f, 0.f);
    float2 v;
    v.x = c.x + beta * (c.x - p.x) - gs * g.x;
    v.y = c.y + beta * (c.y - p.y) - gs * g.y;
    vo[e] = v;
  }
  if (t == 0) {
    if (a.rowflag_prev != nullptr) a.rowflag_prev[row] = fc ? 1 : 0;  // x_k is x_{k-1} next time
    a.rowflag[row] = 0;
    if (row % a.ny == 0) a.planeflag[row / a.ny] = 0;
  }
}

// ---------------------------------------------------------------------------
// Objective partials of a volume: sum(x) and TV3D(x) (forward differences,
// zero past the last index).  One block per 4 rows (z, y).
// ---------------------------------------------------------------------------
constexpr int kObjRows = 4;
constexpr int kObjThreads = 256;

__device__ __forceinline__ void obj_body(const ObjArgs& a, int bx, int) {
  __shared__ double red[2][16];
  if (solve_done(a.st)) return;
  if (a.first_only && a.st != nullptr && a.st->it > 0) return;
  const float* x = a.x0;
  if (a.st != nullptr) {
    // runs before the scalar kernel of the iteration: the iterate is slot it % 3
    x = pick3(a.x0, a.x1, a.x2, a.st->it % 3);
  }
  const int nx = a.nx, ny = a.ny, nz = a.nz;
  const long nrows = (long)ny * nz;
  double s_acc = 0.0, t_acc = 0.0;
  // Each thread takes four consecutive voxels of a row (nx is a multiple of 4;
  // volumes are only 8-byte aligned, so they are read as float2 pairs).  The
  // rows of the block are unrolled so that all their loads are in flight
  // together; rows longer than 4 x kObjThreads take several chunks.
  constexpr int CH = kObjThreads * 4;
  const int i0 = threadIdx.x * 4;
  const int ilast = i0 < nx ? i0 + ((nx - 1 - i0) / CH) * CH : -1;  // this thread's last chunk
  auto ld4 = [](const float* p) {
    const float2 u = *reinterpret_cast<const float2*>(p);
    const float2 w = *reinterpret_cast<const float2*>(p + 2);
    return make_float4(u.x, u.y, w.x, w.y);
  };
  const float4 zero = make_float4(0.f, 0.f, 0.f, 0.f);
  auto reduce4 = [&](int i, float4 v, float vx, float4 vy, float4 vz, bool hy, bool hz) {
    const float a4[5] = {v.x, v.y, v.z, v.w, vx};
    const float b4[4] = {vy.x, vy.y, vy.z, vy.w};
    const float c4[4] = {vz.x, vz.y, vz.z, vz.w};
    float ss = 0.f, tt = 0.f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float gx = (i + k + 1 < nx) ? a4[k + 1] - a4[k] : 0.f;
      const float gy = hy ? b4[k] - a4[k] : 0.f;
      const float gz = (hz && !a.tv2) ? c4[k] - a4[k] : 0.f;
      ss += fabsf(a4[k]);   // ||x||_1 (x >= 0 in the constrained problem, signed otherwise)
      // per-voxel norm in FP32 (relative error ~1e-7), running sums in FP64
      tt += sqrtf(fmaf(gx, gx, fmaf(gy, gy, gz * gz)));
    }
    s_acc += (double)ss;
    t_acc += (double)tt;
  };
  float4 v[kObjRows], vy[kObjRows], vz[kObjRows];
  float vx[kObjRows];
  bool on[kObjRows], hy[kObjRows], hz[kObjRows];
#pragma unroll
  for (int rr = 0; rr < kObjRows; ++rr) {
    const long row = (long)bx * kObjRows + rr;
    on[rr] = row < nrows && ilast >= 0;
    const int z = row < nrows ? (int)(row / ny) : 0, y = row < nrows ? (int)(row % ny) : 0;
    hy[rr] = y + 1 < ny;
    hz[rr] = z + 1 < nz;
    bool f0 = on[rr], fy = on[rr] && hy[rr], fz = on[rr] && hz[rr] && !a.tv2;
    const float* r0 = x + (size_t)(row < nrows ? row : 0) * nx;
    const float* ry = r0 + nx;
    const float* rz = r0 + (size_t)ny * nx;
    if (a.rs.on && on[rr]) {
      // rows from the iterate's store: an absent row is all zero
      const int k = a.st != nullptr ? (a.st->it & 1) : 0;
      r0 = store_row(a.rs, k, (size_t)row);
      ry = fy ? store_row(a.rs, k, (size_t)row + 1) : nullptr;
      rz = fz ? store_row(a.rs, k, (size_t)row + ny) : nullptr;
      f0 = r0 != nullptr;
      fy = ry != nullptr;
      fz = rz != nullptr;
    } else if (a.rowflag != nullptr && on[rr]) {
      f0 = a.rowflag[row] != 0;
      fy = fy && a.rowflag[row + 1] != 0;
      fz = fz && a.rowflag[row + ny] != 0;
    }
    v[rr] = vy[rr] = vz[rr] = zero;
    vx[rr] = 0.f;
    if (!on[rr]) continue;
    for (int i = i0; i <= ilast; i += CH) {
      v[rr] = f0 ? ld4(r0 + i) : zero;
      vx[rr] = (f0 && i + 4 < nx) ? r0[i + 4] : 0.f;
      vy[rr] = fy ? ld4(ry + i) : zero;
      vz[rr] = fz ? ld4(rz + i) : zero;
      if (i != ilast) reduce4(i, v[rr], vx[rr], vy[rr], vz[rr], hy[rr], hz[rr]);
    }
  }
#pragma unroll
  for (int rr = 0; rr < kObjRows; ++rr)
    if (on[rr]) reduce4(ilast, v[rr], vx[rr], vy[rr], vz[rr], hy[rr], hz[rr]);
  s_acc = block_sum<kObjThreads>(s_acc, red[0]);
  __syncthreads();
  t_acc = block_sum<kObjThreads>(t_acc, red[1]);
  if (threadIdx.x == 0) {
    a.psum[bx] = s_acc;
    a.ptv[bx] = t_acc;
  }
}

// ---------------------------------------------------------------------------
// FISTA scalars (one block).
// ---------------------------------------------------------------------------
constexpr int kScalarThreads = 1024;

__device__ __forceinline__ void scalars_body(const ScalarArgs& a, int, int) {
  __shared__ double red[3][16];
  SolveState* st = a.st;
  if (st->done) return;
  double d = 0.0, s = 0.0, t = 0.0;
  for (int i = threadIdx.x; i < a.n_dfit; i += kScalarThreads) d += a.pdfit[i];
  // sum(x_it) and TV(x_it): from the prox that produced x_it, or for x_0 from k_obj
  const bool from_prox = a.qsum != nullptr && st->it > 0;
  const double* ps = from_prox ? a.qsum : a.psum;
  const double* pt = from_prox ? a.qtv : a.ptv;
  const int n_obj = from_prox ? a.n_prox : a.n_obj;
  for (int i = threadIdx.x; i < n_obj; i += kScalarThreads) {
    s += ps[i];
    t += pt[i];
  }
  d = block_sum<kScalarThreads>(d, red[0]);
  __syncthreads();
  s = block_sum<kScalarThreads>(s, red[1]);
  __syncthreads();
  t = block_sum<kScalarThreads>(t, red[2]);
  if (threadIdx.x != 0) return;
  const double F = d + st->l1 * s + st->tv * t;
  const int it = st->it;
  if (it < kHistCap) a.hist[it] = F;
  st->f_cur = F;
  int done = 0;
  if (!isfinite(F)) {
    st->status = RI_ERR_NONFINITE;
    done = 1;
  }
  if (it == 0) st->f_first = F;
  else if (F > 10.0 * st->f_first && F > 0.0) {
    st->status = RI_ERR_NOT_CONVERGED;
    done = 1;
  }
  if (st->f_ref > 0.0) {
    st->gap = (F - st->f_ref) / st->f_ref;
    if (st->gap <= st->gap_tol) {
      st->converged = 1;
      done = 1;
    }
  }
  if (it >= st->max_iters) done = 1;
  if (a.count != nullptr) st->rows_peak = max(st->rows_peak, (int)a.count[it & 1]);   // rows of x_it
  if (a.overflow != nullptr && *a.overflow != 0) {   // a row store ran out of rows (or a wait bound was hit): x_it is incomplete
    st->status = RI_ERR_WORKSPACE_TOO_SMALL;
    st->converged = 0;
    done = 1;
  }
  // slots of this iteration: x_it in it%3, x_{it-1} in (it+2)%3, x_{it+1} -> (it+1)%3
  st->cur = it % 3;
  st->prev = (it + 2) % 3;
  st->next = (it + 1) % 3;
  st->scur = it & 1;
  st->ax_cur = it & 1;
  st->ax_prev = (it + 1) & 1;
  if (done) {
    st->done = 1;
    return;
  }
  double beta = 0.0;
  if (it > 0) {
    const double sn = 0.5 * (1.0 + sqrt(1.0 + 4.0 * st->s * st->s));
    beta = (st->s - 1.0) / sn;
    st->s = sn;
    if (st->restart && F > st->f_prev) {
      st->s = 1.0;
      beta = 0.0;
    }
  }
  st->beta = beta;
  st->f_prev = F;
  st->it = it + 1;
}

__global__ void k_state_init(SolveState* st, StateInit in) {
  SolveState s = {};
  s.it = 0;
  s.done = 0;
  s.converged = 0;
  s.status = RI_OK;
  s.cur = 0; s.prev = 2; s.next = 1;
  s.scur = 0;
  s.rows_peak = 0;
  s.ax_cur = 0; s.ax_prev = 1;
  s.max_iters = in.max_iters;
  s.restart = in.restart;
  s.s = 1.0;
  s.beta = 0.0;
  s.f_prev = 0.0;
  s.f_first = 0.0;
  s.f_cur = 0.0;
  s.gap = __builtin_nan("");
  s.f_ref = in.f_ref;
  s.gap_tol = in.gap_tol;
  s.l1 = in.l1;
  s.tv = in.tv;
  *st = s;
}

// ---------------------------------------------------------------------------
// Utility kernels
// ---------------------------------------------------------------------------
__global__ void k_fill_f32(float* p, size_t n, float v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_u8(uint8_t* p, size_t n, uint8_t v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_copy_f32(float* d, const float* s, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) d[i] = s[i];
}
__global__ void k_copy_final(const float* x0, const float* x1, const float* x2, float* dst, size_t n,
                             const SolveState* st) {
  const float* src = pick3(x0, x1, x2, st->cur);
  if (src == dst) return;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) dst[i] = src[i];
}
__global__ void k_flags_from_x(const float* x, int nx, long nrows, int ny, uint8_t* rowflag, uint8_t* planeflag) {
  const long row = blockIdx.x;
  if (row >= nrows) return;
  int any = 0;
  for (int i = threadIdx.x; i < nx; i += blockDim.x) any |= (x[(size_t)row * nx + i] != 0.f);
  any = __syncthreads_or(any);
  if (threadIdx.x == 0 && any) {
    rowflag[row] = 1;
    planeflag[row / ny] = 1;
  }
}

// Row stores: dense copy of the current store, start, clear of the next store.
__global__ void k_store_expand(RowStores rs, float* dst, size_t n, const SolveState* st) {
  const int k = st->scur;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float* r = store_row(rs, k, i / rs.nx);
    dst[i] = r != nullptr ? r[i % rs.nx] : 0.f;
  }
}

__global__ void k_store_reset(RowStores rs) {
  if (threadIdx.x < 2) rs.count[threadIdx.x] = 0;
  if (threadIdx.x == 2) *rs.overflow = 0;
}

// One block per row: a row with a non-zero value takes a pool row in stores 0
// and 1 (x_0 and x_{-1}); the others are marked absent in both.  x == nullptr
// starts from the zero volume (every row absent).
__global__ void k_store_start(RowStores rs, const float* x, long nrows) {
  const long row = blockIdx.x;
  if (row >= nrows) return;
  const float* src = x != nullptr ? x + (size_t)row * rs.nx : nullptr;
  int any = 0;
  if (src != nullptr)
    for (int i = threadIdx.x; i < rs.nx; i += blockDim.x) any |= (src[i] != 0.f);
  any = __syncthreads_or(any);
  __shared__ int32_t s0, s2;
  if (threadIdx.x == 0) {
    s0 = s2 = -1;
    if (any) {
      const uint32_t a = atomicAdd(&rs.count[0], 1u), b = atomicAdd(&rs.count[1], 1u);
      if (a < rs.cap && b < rs.cap) {
        s0 = (int32_t)a;
        s2 = (int32_t)b;
      } else {
        atomicOr(rs.overflow, 1u);
      }
    }
    rs.slot[0][row] = s0;
    rs.slot[1][row] = s2;
  }
  __syncthreads();
  if (s0 < 0) return;
  float* d0 = rs.pool[0] + (size_t)s0 * rs.nx;
  float* d2 = rs.pool[1] + (size_t)s2 * rs.nx;
  for (int i = threadIdx.x; i < rs.nx; i += blockDim.x) {
    const float v = src[i];
    d0[i] = v;
    d2[i] = v;
  }
}

// Recycle the store of x_{k-1} for x_{k+1}: zero the pool rows it used (every
// pool row not in use stays zero) and mark every row absent; the count is
// reset by a second kernel, after every block has read it.
__global__ void k_store_clear_next(RowStores rs, long nrows, const SolveState* st) {
  if (st->done) return;
  const int k = st->scur ^ 1;
  int32_t* sl = k == 0 ? rs.slot[0] : rs.slot[1];
  float* pl = k == 0 ? rs.pool[0] : rs.pool[1];
  const size_t used = (size_t)min(rs.count[k], rs.cap) * rs.nx;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < used; i += stride) pl[i] = 0.f;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < nrows; i += (long)stride) sl[i] = -1;
}

__global__ void k_store_count_reset(RowStores rs, const SolveState* st) {
  if (st->done) return;
  if (threadIdx.x == 0) rs.count[st->scur ^ 1] = 0;
}

static int grid_for(size_t n) {
  size_t b = (n + 255) / 256;
  return (int)(b > 65536 ? 65536 : (b == 0 ? 1 : b));
}

__global__ void k_scale_f32(float* p, size_t n, float v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] *= v;
}
hipError_t launch_scale_f32(float* p, size_t n, float v, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_f32, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_f32(float* p, size_t n, float v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_u8(uint8_t* p, size_t n, uint8_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u8, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_copy_f32(float* d, const float* src, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_f32, dim3(grid_for(n)), dim3(256), 0, s, d, src, n);
  return hipGetLastError();
}
hipError_t launch_copy_final(const float* x0, const float* x1, const float* x2, float* dst, size_t n,
                             const SolveState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_final, dim3(grid_for(n)), dim3(256), 0, s, x0, x1, x2, dst, n, st);
  return hipGetLastError();
}
hipError_t launch_flags_from_x(const float* x, int nx, int ny, int nz, uint8_t* rowflag, uint8_t* planeflag,
                               hipStream_t s) {
  const long nrows = (long)ny * nz;
  hipLaunchKernelGGL(k_flags_from_x, dim3((unsigned)nrows), dim3(256), 0, s, x, nx, nrows, ny, rowflag, planeflag);
  return hipGetLastError();
}
hipError_t launch_store_expand(const RowStores& rs, float* dst, int ny, int nz, const SolveState* st, hipStream_t s) {
  const size_t n = (size_t)rs.nx * ny * nz;
  hipLaunchKernelGGL(k_store_expand, dim3(grid_for(n)), dim3(256), 0, s, rs, dst, n, st);
  return hipGetLastError();
}
hipError_t launch_store_start(const RowStores& rs, const float* x, int ny, int nz, hipStream_t s) {
  const long nrows = (long)ny * nz;
  // every pool row starts zero; the rows of x_0 are then written whole
  for (int k = 0; k < 2; ++k)
    hipLaunchKernelGGL(k_fill_f32, dim3(grid_for((size_t)rs.cap * rs.nx)), dim3(256), 0, s, rs.pool[k],
                       (size_t)rs.cap * rs.nx, 0.f);
  hipLaunchKernelGGL(k_store_reset, dim3(1), dim3(64), 0, s, rs);
  hipLaunchKernelGGL(k_store_start, dim3((unsigned)nrows), dim3(256), 0, s, rs, x, nrows);
  return hipGetLastError();
}
hipError_t launch_store_clear_next(const RowStores& rs, int ny, int nz, const SolveState* st, hipStream_t s) {
  const long nrows = (long)ny * nz;
  hipLaunchKernelGGL(k_store_clear_next, dim3(grid_for((size_t)nrows * rs.nx)), dim3(256), 0, s, rs, nrows, st);
  hipLaunchKernelGGL(k_store_count_reset, dim3(1), dim3(64), 0, s, rs, st);
  return hipGetLastError();
}
hipError_t launch_state_init(SolveState* st, const StateInit& init, hipStream_t s) {
  hipLaunchKernelGGL(k_state_init, dim3(1), dim3(1), 0, s, st, init);
  return hipGetLastError();
}
// ---------------------------------------------------------------------------
// Lipschitz constant: S(f) = sum_j cos^2(2 pi (c_j + z_j theta(f))) in FP64,
// block maxima over the half-spectrum grid (the full grid is symmetric).
// ---------------------------------------------------------------------------
__global__ void k_lipschitz(PlanTables pt, int m, int ny, int nz, double* pmax) {
  __shared__ double red[256];
  const long n = (long)ny * (m + 1);
  double best = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const double th = pt.theta[i];
    double acc = 0.0;
    for (int j = 0; j < nz; ++j) {
      double ph = fma(pt.zc[j].x, th, pt.zc[j].y);
      ph -= floor(ph);
      const double c = cospi(2.0 * ph);
      acc += c * c;
    }
    best = fmax(best, acc);
  }
  red[threadIdx.x] = best;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) pmax[blockIdx.x] = red[0];
}

hipError_t launch_lipschitz(const PlanTables& pt, int m, int ny, int nz, double* pmax, int* nblocks,
                            hipStream_t s) {
  const long n = (long)ny * (m + 1);
  int nb = (int)((n + 255) / 256);
  if (nb > 1024) nb = 1024;
  *nblocks = nb;
  hipLaunchKernelGGL(k_lipschitz, dim3(nb), dim3(256), 0, s, pt, m, ny, nz, pmax);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Single-frame and batched entry kernels
// ---------------------------------------------------------------------------
__device__ __forceinline__ void batch_find(BatchMap map, int& frame, int& local) {
  const uint32_t b = blockIdx.x;
  int lo = 0, hi = map.n;  // largest f with offs[f] <= b
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (map.offs[mid] <= b) lo = mid;
    else hi = mid;
  }
  frame = lo;
  local = (int)(b - map.offs[lo]);
}

template <class Args>
__device__ __forceinline__ void batch_entry(const Args* __restrict__ args, BatchMap map,
                                            Args& a, int& bx, int& by) {
  int f, lb;
  batch_find(map, f, lb);
  a = args[f];
  bx = lb % a.gx;
  by = lb / a.gx;
}

#define RIHVR_ENTRY_T(NAME, BODY, ARGS, TP, NT)                                                   \
  template <int TP>                                                                               \
  __global__ void __launch_bounds__(NT) NAME(ARGS a) { BODY<TP>(a, blockIdx.x, blockIdx.y); }      \
  template <int TP>                                                                               \
  __global__ void __launch_bounds__(NT) NAME##_b(const ARGS* __restrict__ args,                   \
                                                 BatchMap map) {              \
    ARGS a;                                                                                       \
    int bx, by;                                                                                   \
    batch_entry(args, map, a, bx, by);                                                            \
    BODY<TP>(a, bx, by);                                                                          \
  }

RIHVR_ENTRY_T(k_rows_r2c, rows_r2c_body, RowsR2CArgs, M, kRowsPerBlock(M) * kRowThreads(M))
RIHVR_ENTRY_T(k_rows_c2r, rows_c2r_body, RowsC2RArgs, M, kRowsPerBlock(M) * kRowThreads(M))
RIHVR_ENTRY_T(k_adj_rows, adj_rows_body, AdjRowsArgs, M, kRowsPerBlock(M) * kRowThreads(M))
// Column kernels: adjacent column tiles read the two halves of the same
// 128-byte lines, so their blocks are placed on the same XCD (shared L2).  With
// 8 points per thread the register file is held to 128 VGPRs (4 waves per
// SIMD: two 8-wave blocks per CU); the larger point counts take what they need.
__host__ __device__ constexpr int kColWavesPerSimd(int ny) { return kColP(ny) <= 8 ? 4 : 1; }
#define RIHVR_ENTRY_COLS(NAME, BODY, ARGS, TP, NT)                                                \
  template <int TP>                                                                               \
  __global__ void __launch_bounds__(NT, kColWavesPerSimd(TP)) NAME(ARGS a) {                      \
    const uint32_t t = xcd_tile(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);      \
    BODY<TP>(a, t % gridDim.x, t / gridDim.x);                                                    \
  }                                                                                               \
  template <int TP>                                                                               \
  __global__ void __launch_bounds__(NT, kColWavesPerSimd(TP)) NAME##_b(const ARGS* __restrict__ args, \
                                                                      BatchMap map) {             \
    ARGS a;                                                                                       \
    int bx, by;                                                                                   \
    batch_entry(args, map, a, bx, by);                                                            \
    BODY<TP>(a, bx, by);                                                                          \
  }
RIHVR_ENTRY_COLS(k_fwd_cols, fwd_cols_body, FwdColsArgs, NY, kColW(NY) * (NY / kColP(NY)))
RIHVR_ENTRY_T(k_holo_cols_inv, holo_cols_inv_body, HoloColsInvArgs, NY, kColW(NY) * (NY / kColP(NY)))
RIHVR_ENTRY_COLS(k_adj_cols, adj_cols_body, AdjColsArgs, NY, kColW(NY) * (NY / kColP(NY)))
#undef RIHVR_ENTRY_T
#undef RIHVR_ENTRY_COLS

__global__ void __launch_bounds__(kObjThreads) k_obj(ObjArgs a) { obj_body(a, blockIdx.x, blockIdx.y); }
__global__ void __launch_bounds__(kObjThreads) k_obj_b(const ObjArgs* __restrict__ args,
                                                       BatchMap map) {
  ObjArgs a;
  int bx, by;
  batch_entry(args, map, a, bx, by);
  obj_body(a, bx, by);
}
__global__ void __launch_bounds__(kScalarThreads) k_scalars(ScalarArgs a) { scalars_body(a, 0, 0); }
__global__ void __launch_bounds__(kScalarThreads) k_scalars_b(const ScalarArgs* __restrict__ args,
                                                              BatchMap map) {
  ScalarArgs a;
  int bx, by;
  batch_entry(args, map, a, bx, by);
  scalars_body(a, bx, by);
}

__global__ void k_count_done(const SolveState* const* __restrict__ states, int n, int32_t* out) {
  int c = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) c += states[i]->done != 0;
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  __shared__ int red[16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < (int)(blockDim.x + 63) / 64; ++w) t += red[w];
    *out = t;
  }
}

// ---------------------------------------------------------------------------
// Grids and size dispatch
// ---------------------------------------------------------------------------
#define RIHVR_ROW_SIZES(X) X(8) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) \
  X(12) X(24) X(48) X(96) X(192) X(384) X(768)
#define RIHVR_COL_SIZES(X) X(16) X(32) X(64) X(128) X(256) X(512) X(1024) X(2048) \
  X(24) X(48) X(96) X(192) X(384) X(768) X(1536)

dim3 grid_rows(int m, int nrows) {
  const int r = kRowsPerBlock(m);
  return dim3((nrows + r - 1) / r);
}
dim3 grid_cols(int ny, int m, int nchunk) {
  const int w = kColW(ny);
  return dim3((m + w - 1) / w, nchunk);
}
static int row_threads(int m) { return kRowsPerBlock(m) * kRowThreads(m); }
static int col_threads(int ny) { return kColW(ny) * (ny / kColP(ny)); }

#define RIHVR_DISPATCH(SIZES, VAR, SINGLE_OR_BATCH)                                          \
  switch (VAR) {                                                                             \
    SIZES(SINGLE_OR_BATCH)                                                                   \
    default: return hipErrorInvalidValue;                                                    \
  }

hipError_t launch_rows_r2c(int m, RowsR2CArgs a, hipStream_t s) {
  const dim3 g = grid_rows(m, a.nrows);
  a.gx = g.x; a.gy = g.y;
#define C(M) case M: hipLaunchKernelGGL(k_rows_r2c<M>, g, dim3(row_threads(M)), 0, s, a); return hipGetLastError();
  RIHVR_DISPATCH(RIHVR_ROW_SIZES, m, C)
#undef C
}
hipError_t launch_rows_r2c_batched(int m, const RowsR2CArgs* args, BatchMap map, int nb, hipStream_t s) {
#define C(M) case M: hipLaunchKernelGGL(k_rows_r2c_b<M>, dim3(nb), dim3(row_threads(M)), 0, s, args, map); return hipGetLastError();
  RIHVR_DISPATCH(RIHVR_ROW_SIZES, m, C)
#undef C
}
hipError_t launch_rows_c2r(int m, RowsC2RArgs a, hipStream_t s) {
  const dim3 g = grid_rows(m, a.nrows);
  a.gx = g.x; a.gy = g.y;
#define C(M) case M: hipLaunchKernelGGL(k_rows_c2r<M>, g, dim3(row_threads(M)), 0, s, a); return hipGetLastError();
  RIHVR_DISPATCH(RIHVR_ROW_SIZES, m, C)
#undef C
}
hipError_t launch_rows_c2r_batched(int m, const RowsC2RArgs* args, BatchMap map, int nb, hipStream_t s) {
#define C(M) case M: hipLaunchKernelGGL(k_rows_c2r_b<M>, dim3(nb), dim3(row_threads(M)), 0, s, args, map); return hipGetLastError();
  RIHVR_DISPATCH(RIHVR_ROW_SIZES, m, C)
#undef C
}
hipError_t launch_adj_rows(int m, AdjRowsArgs a, hipStream_t s) {
  const dim3 g = grid_rows(m, a.nrows);
  a.gx = g.x; a.gy = g.y;
#define C(M) case M: hipLaunchKernelGGL(k_adj_rows<M>, g, dim3(row_threads(M)), 0, s, a); return hipGetLastError();
  RIHVR_DISPATCH(RIHVR_ROW_SIZES, m, C)
#undef C
}
hipError_t launch_adj_rows_batched(int m, const AdjRowsArgs* args, BatchMap map, int nb, hipStream_t s) {
#define C(M) case M: hipLaunchKernelGGL(k_adj_rows_b<M>, dim3(nb), dim3(row_threads(M)), 0, s, args, map); return hipGetLastError();
  RIHVR_DISPATCH(RIHVR_ROW_SIZES, m, C)
#undef C
}
hipError_t launch_fwd_cols(int ny, int nchunk, FwdColsArgs a, hipStream_t s) {
  const dim3 g = grid_cols(ny, a.m, nchunk);
  a.gx = g.x; a.gy = g.y;
#define C(NY) case NY: hipLaunchKernelGGL(k_fwd_cols<NY>, g, dim3(col_threads(NY)), 0, s, a); return hipGetLastError();
  RIHVR_DISPATCH(RIHVR_COL_SIZES, ny, C)
#undef C
}
hipError_t launch_fwd_cols_batched(int ny, const FwdColsArgs* args, BatchMap map, int nb, hipStream_t s) {
#define C(NY) case NY: hipLaunchKernelGGL(k_fwd_cols_b<NY>, dim3(nb), dim3(col_threads(NY)), 0, s, args, map); return hipGetLastError();
  RIHVR_DISPATCH(RIHVR_COL_SIZES, ny, C)
#undef C
}
hipError_t launch_holo_cols_inv(int ny, HoloColsInvArgs a, hipStream_t s) {
  const dim3 g = grid_cols(ny, a.m, 1);
  a.gx = g.x; a.gy = g.y;
#define C(NY) case NY: hipLaunchKernelGGL(k_holo_cols_inv<NY>, g, dim3(col_threads(NY)), 0, s, a); return hipGetLastError();
  RIHVR_DISPATCH(RIHVR_COL_SIZES, ny, C)
#undef C
}
hipError_t launch_holo_cols_inv_batched(int ny, const HoloColsInvArgs* args, BatchMap map, int nb,
                                        hipStream_t s) {
#define C(NY) case NY: hipLaunchKernelGGL(k_holo_cols_inv_b<NY>, dim3(nb), dim3(col_threads(NY)), 0, s, args, map); return hipGetLastError();
  RIHVR_DISPATCH(RIHVR_COL_SIZES, ny, C)
#undef C
}
hipError_t launch_adj_cols(int ny, int nchunk, AdjColsArgs a, hipStream_t s) {
  const dim3 g = grid_cols(ny, a.m, nchunk);
  a.gx = g.x; a.gy = g.y;
#define C(NY) case NY: hipLaunchKernelGGL(k_adj_cols<NY>, g, dim3(col_threads(NY)), 0, s, a); return hipGetLastError();
  RIHVR_DISPATCH(RIHVR_COL_SIZES, ny, C)
#undef C
}
hipError_t launch_adj_cols_batched(int ny, const AdjColsArgs* args, BatchMap map, int nb, hipStream_t s) {
#define C(NY) case NY: hipLaunchKernelGGL(k_adj_cols_b<NY>, dim3(nb), dim3(col_threads(NY)), 0, s, args, map); return hipGetLastError();
  RIHVR_DISPATCH(RIHVR_COL_SIZES, ny, C)
#undef C
}

dim3 grid_obj(int nx, int ny, int nz) {
  (void)nx;
  return dim3((unsigned)(((long)ny * nz + kObjRows - 1) / kObjRows));
}
int obj_blocks(int nx, int ny, int nz) { return (int)grid_obj(nx, ny, nz).x; }
hipError_t launch_obj(ObjArgs a, hipStream_t s) {
  const dim3 g = grid_obj(a.nx, a.ny, a.nz);
  a.gx = g.x; a.gy = 1;
  hipLaunchKernelGGL(k_obj, g, dim3(kObjThreads), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_obj_batched(const ObjArgs* args, BatchMap map, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_obj_b, dim3(nb), dim3(kObjThreads), 0, s, args, map);
  return hipGetLastError();
}
hipError_t launch_scalars(ScalarArgs a, hipStream_t s) {
  a.gx = 1; a.gy = 1;
  hipLaunchKernelGGL(k_scalars, dim3(1), dim3(kScalarThreads), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_scalars_batched(const ScalarArgs* args, BatchMap map, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_scalars_b, dim3(nb), dim3(kScalarThreads), 0, s, args, map);
  return hipGetLastError();
}
hipError_t launch_count_done(const SolveState* const* states, int n, int32_t* out, hipStream_t s) {
  hipLaunchKernelGGL(k_count_done, dim3(1), dim3(1024), 0, s, states, n, out);
  return hipGetLastError();
}

}  // namespace rihvr
