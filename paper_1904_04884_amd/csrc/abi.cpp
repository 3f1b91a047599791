// C ABI of the library: argument validation, plans (FP64 tables), workspace
// layouts and the host side of the FISTA solve (kernel sequencing, HIP graph
// replay, stop-flag polling, phase timing).
#include <hip/hip_runtime.h>

#include <unistd.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "rihvr_internal.h"

using namespace rihvr;

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
static thread_local char g_last_error[512] = "";

static ri_status fail(ri_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
  va_end(ap);
  return st;
}

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(RI_ERR_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
  } while (0)

extern "C" const char* ri_status_string(ri_status s) {
  switch (s) {
    case RI_OK: return "ok";
    case RI_ERR_INVALID_ARG: return "invalid argument";
    case RI_ERR_UNSUPPORTED_SIZE: return "unsupported size";
    case RI_ERR_OUT_OF_MEMORY: return "out of memory";
    case RI_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case RI_ERR_HIP: return "HIP runtime error";
    case RI_ERR_NONFINITE: return "non-finite objective";
    case RI_ERR_NOT_CONVERGED: return "objective diverged";
  }
  return "unknown status";
}

extern "C" const char* ri_last_error(void) { return g_last_error; }

namespace rihvr {
ri_status set_error(ri_status st, const char* msg) { return fail(st, "%s", msg); }
}  // namespace rihvr

// ---------------------------------------------------------------------------
// Plan
// ---------------------------------------------------------------------------
struct GraphCache {
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  // key: everything that is baked into the captured launches
  const void* ws = nullptr;
  const void* b = nullptr;
  const void* x = nullptr;
  double step = 0, l1 = 0, tv = 0;
  int inner = -1, dense = -1, nonneg = -1, warm = -1;
  double store_frac = -1.0;
};

struct ri_plan {
  ri_geometry g{};
  int m = 0;                 // nx / 2
  int device = 0;
  int cus = 0;               // compute units of the device
  double lipschitz = 0.0;
  double* theta = nullptr;   // device [ny][m+1]
  double2* zc = nullptr;     // device [nz]
  float2* tw_row = nullptr;  // device [nx]
  float2* tw_col = nullptr;  // device [ny]
  int32_t* host_flag = nullptr;  // pinned, for stop polling
  hipStream_t capture = nullptr;
  GraphCache gc;
  ri_tuning tune{kTvDefaultLevels, kTvDefaultBlocks, kColDefaultBlocks};
  double store_frac = 0.0;   // > 0: row-compressed iterates with room for this fraction of rows
  bool cplx = false;         // complex object: g.nz counts the planes of both parts
  ri_dtype dtype = RI_F32;
  int dual_planes = 0;       // RI_TV2D: planes whose TV dual is held at a time (0: the volume)
  double2* tw64x = nullptr;  // FP64 plans: exp(-2 pi i k / nx), k < nx
  double2* tw64y = nullptr;  //             exp(-2 pi i k / ny), k < ny
  PlanTables tables() const { return PlanTables{theta, zc, tw_row, tw_col}; }
};


static bool supported_nx(int nx) { return nx >= 16 && nx <= 2048 && nx % 2 == 0 && fft_len_supported(nx / 2); }
static bool supported_ny(int ny) { return ny >= 16 && ny <= 2048 && fft_len_supported(ny); }

static void free_plan(ri_plan* p) {
  if (!p) return;
  if (p->gc.exec) hipGraphExecDestroy(p->gc.exec);
  if (p->gc.graph) hipGraphDestroy(p->gc.graph);
  if (p->capture) hipStreamDestroy(p->capture);
  if (p->theta) hipFree(p->theta);
  if (p->zc) hipFree(p->zc);
  if (p->tw_row) hipFree(p->tw_row);
  if (p->tw_col) hipFree(p->tw_col);
  if (p->tw64x) hipFree(p->tw64x);
  if (p->tw64y) hipFree(p->tw64y);
  if (p->host_flag) hipHostFree(p->host_flag);
  delete p;
}

static void drop_graph(ri_plan* p) {
  if (p->gc.exec) hipGraphExecDestroy(p->gc.exec);
  if (p->gc.graph) hipGraphDestroy(p->gc.graph);
  p->gc = GraphCache{};
}

static void twiddles(int n, std::vector<float2>& out) {
  out.resize(n);
  for (int k = 0; k < n; ++k) {
    // exp(-2 pi i k / n) from the FP64 angle, rounded once to FP32
    const double a = 2.0 * M_PI * (double)k / (double)n;
    out[k] = make_float2((float)std::cos(a), (float)(-std::sin(a)));
  }
}

static ri_status validate_geometry(const ri_geometry* g) {
  if (!g) return fail(RI_ERR_INVALID_ARG, "geometry is NULL");
  if (!supported_nx(g->nx) || !supported_ny(g->ny))
    return fail(RI_ERR_UNSUPPORTED_SIZE, "nx=%d ny=%d: sizes must be 2^a or 3*2^a in [16, 2048]", g->nx, g->ny);
  if (g->nz < 1) return fail(RI_ERR_INVALID_ARG, "nz=%d must be >= 1", g->nz);
  if (!(g->pixel_um > 0) || !(g->wavelength_um > 0) || !std::isfinite(g->z0_um) || !std::isfinite(g->dz_um))
    return fail(RI_ERR_INVALID_ARG, "pixel and wavelength must be > 0, z0 and dz finite");
  // every grid frequency must propagate: max f^2 = 1/(4 px^2) * 2 < 1/lambda^2
  const double fmax2 = 0.5 / (g->pixel_um * g->pixel_um);
  if (!(fmax2 < 1.0 / (g->wavelength_um * g->wavelength_um)))
    return fail(RI_ERR_INVALID_ARG, "pixel %.4g um <= lambda/sqrt(2): evanescent frequencies are not supported",
                g->pixel_um);
  if (g->flags & ~(RI_NO_CARRIER | RI_TV2D | RI_TV_FGP | RI_TV_DUAL_BF16 | RI_COMPLEX))
    return fail(RI_ERR_INVALID_ARG, "unknown geometry flags 0x%x", g->flags);
  if ((g->flags & RI_COMPLEX) && (g->flags & (RI_TV_FGP | RI_TV_DUAL_BF16)))
    return fail(RI_ERR_INVALID_ARG, "RI_COMPLEX plans take neither RI_TV_FGP nor RI_TV_DUAL_BF16");
  if ((g->flags & RI_COMPLEX) && g->nz > (1 << 30))
    return fail(RI_ERR_INVALID_ARG, "nz=%d too large for a complex plan", g->nz);
  return RI_OK;
}

extern "C" ri_status ri_plan_create(const ri_geometry* g, ri_dtype dtype, ri_plan** out) {
  if (!out) return fail(RI_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (dtype != RI_F32 && dtype != RI_F64) return fail(RI_ERR_INVALID_ARG, "unknown dtype %d", (int)dtype);
  ri_status vs = validate_geometry(g);
  if (vs != RI_OK) return vs;
  if (dtype == RI_F64 && (g->flags & (RI_TV_FGP | RI_TV_DUAL_BF16)))
    return fail(RI_ERR_INVALID_ARG, "RI_F64 plans take neither RI_TV_FGP nor RI_TV_DUAL_BF16");
  ri_plan* p = new ri_plan();
  p->g = *g;
  p->dtype = dtype;
  p->m = g->nx / 2;
  // A complex object is two real volumes (real parts, imaginary parts): the
  // plan covers 2 nz planes, the second nz with the carrier a quarter cycle on
  // (i H_j), so A acting on the imaginary parts is Re(IFFT2(FFT2(i x_j) H_j)).
  p->cplx = (g->flags & RI_COMPLEX) != 0;
  if (p->cplx) p->g.nz = 2 * g->nz;
  const int nx = g->nx, ny = g->ny, nz = p->g.nz, m = p->m;
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) { free_plan(p); return fail(RI_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e)); }
  e = hipDeviceGetAttribute(&p->cus, hipDeviceAttributeMultiprocessorCount, p->device);
  if (e != hipSuccess) { free_plan(p); return fail(RI_ERR_HIP, "hipDeviceGetAttribute: %s", hipGetErrorString(e)); }

  // theta(f) = sqrt(1/lambda^2 - f^2) - 1/lambda = -f^2 / (sqrt(1/lambda^2 - f^2) + 1/lambda)
  const double il = 1.0 / g->wavelength_um;
  std::vector<double> theta((size_t)ny * (m + 1));
  for (int ky = 0; ky < ny; ++ky) {
    const double fy = (double)(ky < (ny + 1) / 2 ? ky : ky - ny) / (ny * g->pixel_um);
    for (int kx = 0; kx <= m; ++kx) {
      const double fx = (double)(kx < m ? kx : -m) / (nx * g->pixel_um);
      const double f2 = fx * fx + fy * fy;
      theta[(size_t)ky * (m + 1) + kx] = -f2 / (std::sqrt(il * il - f2) + il);
    }
  }
  std::vector<double2> zc(nz);
  for (int j = 0; j < nz; ++j) {
    const int jp = p->cplx ? j % g->nz : j;              // plane of the part
    const double z = g->z0_um + g->dz_um * jp;
    double c = 0.0;
    if (!(g->flags & RI_NO_CARRIER)) {
      const double t = z / g->wavelength_um;
      c = t - std::floor(t);
    }
    if (p->cplx && j >= g->nz) {
      c += 0.25;
      c -= std::floor(c);
    }
    zc[j] = make_double2(z, c);
  }
  std::vector<float2> twr, twc;
  twiddles(nx, twr);
  twiddles(ny, twc);

#define PLAN_TRY(expr)                                                                        \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) {                                                                   \
      free_plan(p);                                                                           \
      return fail(e_ == hipErrorOutOfMemory ? RI_ERR_OUT_OF_MEMORY : RI_ERR_HIP, "%s: %s", #expr, \
                  hipGetErrorString(e_));                                                     \
    }                                                                                         \
  } while (0)
  PLAN_TRY(hipMalloc(&p->theta, theta.size() * sizeof(double)));
  PLAN_TRY(hipMalloc(&p->zc, zc.size() * sizeof(double2)));
  PLAN_TRY(hipMalloc(&p->tw_row, twr.size() * sizeof(float2)));
  PLAN_TRY(hipMalloc(&p->tw_col, twc.size() * sizeof(float2)));
  PLAN_TRY(hipHostMalloc(&p->host_flag, 64 * sizeof(int32_t)));
  PLAN_TRY(hipMemcpy(p->theta, theta.data(), theta.size() * sizeof(double), hipMemcpyHostToDevice));
  PLAN_TRY(hipMemcpy(p->zc, zc.data(), zc.size() * sizeof(double2), hipMemcpyHostToDevice));
  PLAN_TRY(hipMemcpy(p->tw_row, twr.data(), twr.size() * sizeof(float2), hipMemcpyHostToDevice));
  PLAN_TRY(hipMemcpy(p->tw_col, twc.data(), twc.size() * sizeof(float2), hipMemcpyHostToDevice));
  PLAN_TRY(hipStreamCreateWithFlags(&p->capture, hipStreamNonBlocking));
  if (dtype == RI_F64) {
    auto tw64 = [](int n, std::vector<double2>& out) {
      out.resize(n);
      for (int k = 0; k < n; ++k) {
        const double a = 2.0 * M_PI * (double)k / (double)n;
        out[k] = make_double2(std::cos(a), -std::sin(a));
      }
    };
    std::vector<double2> t64x, t64y;
    tw64(nx, t64x);
    tw64(ny, t64y);
    PLAN_TRY(hipMalloc(&p->tw64x, t64x.size() * sizeof(double2)));
    PLAN_TRY(hipMalloc(&p->tw64y, t64y.size() * sizeof(double2)));
    PLAN_TRY(hipMemcpy(p->tw64x, t64x.data(), t64x.size() * sizeof(double2), hipMemcpyHostToDevice));
    PLAN_TRY(hipMemcpy(p->tw64y, t64y.data(), t64y.size() * sizeof(double2), hipMemcpyHostToDevice));
  }

  // ||A||^2 = max over the grid of sum_j cos^2(phase_j) (FP64, on the device)
  double* pmax = nullptr;
  PLAN_TRY(hipMalloc(&pmax, 1024 * sizeof(double)));
  int nb = 0;
  hipError_t le = launch_lipschitz(p->tables(), m, ny, nz, pmax, &nb, p->capture);
  std::vector<double> hmax(1024, 0.0);
  if (le == hipSuccess) le = hipStreamSynchronize(p->capture);
  if (le == hipSuccess) le = hipMemcpy(hmax.data(), pmax, nb * sizeof(double), hipMemcpyDeviceToHost);
  hipFree(pmax);
  if (le != hipSuccess) {
    free_plan(p);
    return fail(RI_ERR_HIP, "Lipschitz kernel: %s", hipGetErrorString(le));
  }
  p->lipschitz = *std::max_element(hmax.begin(), hmax.begin() + nb);
  if (!(p->lipschitz > 0.0)) {
    free_plan(p);
    return fail(RI_ERR_INVALID_ARG, "||A||^2 = 0 for this geometry");
  }
  *out = p;
  return RI_OK;
#undef PLAN_TRY
}

extern "C" ri_status ri_plan_destroy(ri_plan* p) {
  if (!p) return fail(RI_ERR_INVALID_ARG, "plan is NULL");
  free_plan(p);
  return RI_OK;
}

extern "C" ri_status ri_plan_lipschitz(const ri_plan* p, double* out) {
  if (!p || !out) return fail(RI_ERR_INVALID_ARG, "NULL argument");
  *out = p->lipschitz;
  return RI_OK;
}

// ---------------------------------------------------------------------------
// Workspace layouts
// ---------------------------------------------------------------------------
struct Layout {
  size_t total = 0;
  size_t vol1 = 0, vol2 = 0, pa[3] = {0, 0, 0}, pb[3] = {0, 0, 0};  // volumes (float; duals float or bf16)
  size_t pa2[3] = {0, 0, 0}, pb2[3] = {0, 0, 0};                   // FGP: second dual of each set
  size_t stage = 0;                                                 // in-place prox with bf16 duals
  size_t pool[2] = {0, 0}, slot[2] = {0, 0}, count = 0, overflow = 0;   // row-compressed iterates
  uint32_t cap = 0;                                                 // pool rows per store (0: dense)
  size_t spec = 0, gp = 0, gi = 0, th = 0;                 // spectra (float2)
  size_t ax0 = 0, ax1 = 0;                                 // holograms (float)
  size_t rowflag = 0, planeflag = 0, rowflag_prev = 0;     // bytes
  size_t pdfit = 0, psum = 0, ptv = 0, qsum = 0, qtv = 0, hist = 0;  // doubles
  size_t state = 0;
  int nchunk = 1, ppc = 1;
  int n_dfit = 0, n_obj = 0, n_prox = 0;  // n_prox: bound over every TV tuning
};

static size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// Candidate launch shapes of the autotuner (distinct grids only are timed).
static const int kTvBlockCands[] = {256, 512, 768, 1536, 3072, 6144};
static const int kColBlockCands[] = {128, 256, 512, 1024, 2048};
static const int kColTuneMax = 2048;

// Planes per chunk of the column transforms: the z-range is cut until the
// column kernels hold about `col_blocks` blocks.
static void chunking(const ri_plan* p, int col_blocks, int* nchunk, int* ppc) {
  const int W = col_tile_width(p->g.ny);
  const int tiles = (p->m + W - 1) / W;
  int want = std::max(1, (col_blocks + tiles - 1) / tiles);
  want = std::min(want, p->g.nz);
  const int per = (p->g.nz + want - 1) / want;
  *ppc = per;
  *nchunk = (p->g.nz + per - 1) / per;
}

// Pool rows of a row store: the requested fraction of the volume's rows (a
// row is allocated once, by the first segment that holds a non-zero value);
// a fraction k / rows gives exactly k rows despite its rounding.
static uint32_t store_cap(const ri_plan* p) {
  const double rows = (double)p->g.ny * p->g.nz;
  return (uint32_t)std::max(1.0, std::min(rows, std::ceil(p->store_frac * rows - 1e-6)));
}

// The grouped per-plane prox applies (RI_TV2D plans with a dual of fewer
// planes than the volume).
static bool plane_group(const ri_plan* p) {
  return (p->g.flags & RI_TV2D) && p->dual_planes > 0 && p->dual_planes < p->g.nz && p->dtype == RI_F32 && !p->cplx;
}

struct Layout64 {
  size_t X = 0, S = 0, hol = 0, y = 0, xp = 0, v = 0, p[3] = {0, 0, 0}, p2[3] = {0, 0, 0}, part = 0, psum = 0,
         ptv = 0;
  int nblk = 0;
  size_t total = 0;
};

// Workspace of an FP64 plan: every plane's complex spectrum and a hologram
// spectrum (A, A^T), the prox's two dual sets, the solver's y, x_{k-1} (then
// x_{k+1}), v, a hologram and per-block partials.  Volumes hold both parts.
static Layout64 layout64(const ri_plan* p, ri_op op) {
  Layout64 L;
  const size_t nx = p->g.nx, ny = p->g.ny, nzp = p->g.nz;
  const size_t vol = nx * ny * nzp * sizeof(double), np = nx * ny;
  size_t off = 256;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  if (op == RI_OP_FORWARD || op == RI_OP_ADJOINT || op == RI_OP_SOLVE) {
    L.X = take(2 * vol);
    L.S = take(np * sizeof(double2));
  }
  if (op == RI_OP_PROX || op == RI_OP_SOLVE) {
    const int nc = (p->g.flags & RI_TV2D) ? 2 : 3;
    for (int k = 0; k < nc; ++k) L.p[k] = take(vol);
    for (int k = 0; k < nc; ++k) L.p2[k] = take(vol);
  }
  if (op == RI_OP_SOLVE) {
    L.hol = take(np * sizeof(double));
    L.y = take(vol);
    L.xp = take(vol);
    L.v = take(vol);
    L.nblk = 1024;
    L.part = take((size_t)L.nblk * sizeof(double));
    L.psum = take((size_t)L.nblk * sizeof(double));
    L.ptv = take((size_t)L.nblk * sizeof(double));
  }
  L.total = off;
  return L;
}

static Layout make_layout(const ri_plan* p, ri_op op, int col_blocks = 0, bool dense_iterates = false) {
  if (p->dtype == RI_F64) {   // only the size is used; the FP64 entry points take layout64
    Layout L64;
    L64.total = layout64(p, op).total;
    return L64;
  }
  if (op == RI_OP_AUTOTUNE) return make_layout(p, RI_OP_SOLVE, kColTuneMax, true);  // room for every candidate
  Layout L;
  const size_t nx = p->g.nx, ny = p->g.ny, nz = p->g.nz, m = p->m;
  const size_t vol = nx * ny * nz * sizeof(float);
  const size_t spec = m * ny * nz * sizeof(float2);
  const size_t hspec = m * ny * sizeof(float2);
  chunking(p, col_blocks > 0 ? col_blocks : p->tune.col_blocks, &L.nchunk, &L.ppc);
  size_t off = 256;  // slack so the base can be aligned up
  // Successive buffers are staggered by 37 x 256 bytes (cycling over 16): the
  // volumes are powers of two in size, and buffers a whole number of GiB apart
  // send the same-index accesses of kernels that stream several of them at once
  // (the TV pass reads v and three dual planes and writes three) to the same
  // memory channels.  Any stagger that is not a multiple of 2 MiB helps; this
  // one made the prox 5 % faster at 1024^2 x 256.
  int nbuf = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes) + (size_t)(++nbuf % 16) * 37 * 256;
    return o;
  };
  if (op == RI_OP_FORWARD || op == RI_OP_SOLVE) {
    L.spec = take(spec);
    L.gp = take((size_t)L.nchunk * hspec);
    L.gi = take(hspec);
  }
  if (op == RI_OP_ADJOINT || op == RI_OP_SOLVE) {
    if (op == RI_OP_ADJOINT) L.spec = take(spec);
    L.th = take(hspec);
  }
  if (op == RI_OP_PROX || op == RI_OP_SOLVE) {
    // dual components: x, y (and z for the 3D TV); the per-plane 2D TV has no z
    // dual.  FGP keeps two duals per set (r and p); bf16 duals take half the bytes.
    const int nc = (p->g.flags & RI_TV2D) ? 2 : 3;
    // the grouped per-plane prox holds its dual for dual_planes planes only
    const size_t dplanes = plane_group(p) ? (size_t)p->dual_planes : nz;
    const size_t dvol = ((p->g.flags & RI_TV_DUAL_BF16) ? nx * ny * dplanes * 2 : nx * ny * dplanes * 4);
    for (int k = 0; k < nc; ++k) L.pa[k] = take(dvol);
    for (int k = 0; k < nc; ++k) L.pb[k] = take(dvol);
    if (p->g.flags & RI_TV_FGP) {
      for (int k = 0; k < nc; ++k) L.pa2[k] = take(dvol);
      for (int k = 0; k < nc; ++k) L.pb2[k] = take(dvol);
    }
    if (op == RI_OP_PROX && (p->g.flags & RI_TV_DUAL_BF16)) L.stage = take(vol);
  }
  if (op == RI_OP_SOLVE) {
    if (p->store_frac > 0.0 && !dense_iterates) {
      // x_k, x_{k-1}, x_{k+1} in row stores; the caller's x_inout holds the
      // dense gradient-step output v during the solve
      L.cap = store_cap(p);
      for (int k = 0; k < 2; ++k) L.pool[k] = take((size_t)L.cap * nx * sizeof(float));
      for (int k = 0; k < 2; ++k) L.slot[k] = take(ny * nz * sizeof(int32_t));
      L.count = take(2 * sizeof(uint32_t));
      L.overflow = take(sizeof(uint32_t));
    } else {
      L.vol1 = take(vol);
      L.vol2 = take(vol);
    }
    L.ax0 = take(nx * ny * sizeof(float));
    L.ax1 = take(nx * ny * sizeof(float));
    L.rowflag = take(ny * nz);
    L.rowflag_prev = take(ny * nz);
    L.planeflag = take(nz);
    L.n_dfit = (int)((ny + rows_per_block((int)m) - 1) / rows_per_block((int)m));
    L.n_obj = obj_blocks((int)nx, (int)ny, (int)nz);
    L.pdfit = take((size_t)L.n_dfit * sizeof(double));
    L.psum = take((size_t)L.n_obj * sizeof(double));
    L.ptv = take((size_t)L.n_obj * sizeof(double));
    L.n_prox = plane_group(p) ? tv_group_blocks_bound((int)nx, (int)ny, (int)nz, p->dual_planes, p->cus)
                              : tv_blocks_bound((int)nx, (int)ny, (int)nz, p->cus);
    L.qsum = take((size_t)L.n_prox * sizeof(double));
    L.qtv = take((size_t)L.n_prox * sizeof(double));
    L.hist = take((size_t)kHistCap * sizeof(double));
    L.state = take(sizeof(SolveState));
  }
  L.total = off;
  return L;
}

extern "C" ri_status ri_workspace_size_op(const ri_plan* p, ri_op op, size_t* bytes) {
  if (!p || !bytes) return fail(RI_ERR_INVALID_ARG, "NULL argument");
  if (op < RI_OP_FORWARD || op > RI_OP_AUTOTUNE) return fail(RI_ERR_INVALID_ARG, "unknown op %d", (int)op);
  *bytes = make_layout(p, op).total;
  return RI_OK;
}

extern "C" ri_status ri_workspace_size(const ri_plan* p, size_t* bytes) {
  if (!p || !bytes) return fail(RI_ERR_INVALID_ARG, "NULL argument");
  size_t n = 0;
  for (int op = RI_OP_FORWARD; op <= RI_OP_AUTOTUNE; ++op) n = std::max(n, make_layout(p, (ri_op)op).total);
  *bytes = n;
  return RI_OK;
}

template <class T>
static T* at(void* ws, size_t off) {
  const uintptr_t base = ((uintptr_t)ws + 255) & ~(uintptr_t)255;
  return reinterpret_cast<T*>(base + off - 256);
}

static bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return x < y + nb && y < x + na;
}

static ri_status check_common(ri_plan* p, const void* in, const void* out, void* ws, size_t ws_bytes, ri_op op,
                              size_t in_bytes, size_t out_bytes) {
  if (!p) return fail(RI_ERR_INVALID_ARG, "plan is NULL");
  if (!in || !out) return fail(RI_ERR_INVALID_ARG, "input or output pointer is NULL");
  if (((uintptr_t)in & 7) || ((uintptr_t)out & 7))
    return fail(RI_ERR_INVALID_ARG, "input and output must be 8-byte aligned");
  const size_t need = make_layout(p, op).total;
  if (!ws) return fail(RI_ERR_INVALID_ARG, "workspace is NULL (needs %zu bytes)", need);
  if (ws_bytes < need) return fail(RI_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes < %zu required", ws_bytes, need);
  if (overlaps(ws, ws_bytes, in, in_bytes) || overlaps(ws, ws_bytes, out, out_bytes))
    return fail(RI_ERR_INVALID_ARG, "workspace overlaps an argument");
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != p->device) return fail(RI_ERR_INVALID_ARG, "plan belongs to device %d, current device is %d", p->device, dev);
  return RI_OK;
}

// Dual buffers and inner-solver options of a prox from the plan and a layout.
static void prox_duals(const ri_plan* p, const Layout& L, void* ws, ProxArgs* a) {
  for (int k = 0; k < 3; ++k) {
    a->pa[k] = at<float>(ws, L.pa[k]);
    a->pb[k] = at<float>(ws, L.pb[k]);
    a->pa2[k] = at<float>(ws, L.pa2[k]);
    a->pb2[k] = at<float>(ws, L.pb2[k]);
  }
  a->tv2 = (p->g.flags & RI_TV2D) ? 1 : 0;
  a->dual_bf16 = (p->g.flags & RI_TV_DUAL_BF16) ? 1 : 0;
  a->fgp = (p->g.flags & RI_TV_FGP) ? 1 : 0;
  a->cus = p->cus;
  a->group_planes = plane_group(p) ? p->dual_planes : 0;
}

// ---------------------------------------------------------------------------
// Operators
// ---------------------------------------------------------------------------
static hipError_t enqueue_forward(ri_plan* p, const Layout& L, void* ws, const float* x, float* out,
                                  hipStream_t s) {
  const PlanTables pt = p->tables();
  const int ny = p->g.ny, nz = p->g.nz, m = p->m;
  RowsR2CArgs ra{};
  ra.x = x;
  ra.out = at<float2>(ws, L.spec);
  ra.nrows = ny * nz;
  ra.mode = 0;
  ra.pt = pt;
  hipError_t e = launch_rows_r2c(m, ra, s);
  if (e != hipSuccess) return e;
  FwdColsArgs fa{};
  fa.t = at<float2>(ws, L.spec);
  fa.gp = at<float2>(ws, L.gp);
  fa.m = m;
  fa.nz = nz;
  fa.planes_per_chunk = L.ppc;
  fa.pt = pt;
  e = launch_fwd_cols(ny, L.nchunk, fa, s);
  if (e != hipSuccess) return e;
  HoloColsInvArgs ha{};
  ha.gp = at<float2>(ws, L.gp);
  ha.gi = at<float2>(ws, L.gi);
  ha.m = m;
  ha.nchunk = L.nchunk;
  ha.pt = pt;
  e = launch_holo_cols_inv(ny, ha, s);
  if (e != hipSuccess) return e;
  RowsC2RArgs ca{};
  ca.in = at<float2>(ws, L.gi);
  ca.nrows = ny;
  ca.out = out;
  ca.mode = 0;
  ca.scale = (float)(1.0 / ((double)p->g.nx * ny));
  ca.pt = pt;
  return launch_rows_c2r(m, ca, s);
}

// ---------------------------------------------------------------------------
// FP64 plans: the same operator from the same FP64 tables, computed plainly in
// double (f64.hip), with the unfused gradient-projection prox (cplx.hip) and a
// FISTA loop driven from the host (scalars, objective and stop in FP64 on the
// host; no graph).
// ---------------------------------------------------------------------------
static size_t elem_bytes(const ri_plan* p) { return p->dtype == RI_F64 ? sizeof(double) : sizeof(float); }

static Plan64Tables tables64(const ri_plan* p) {
  return Plan64Tables{p->theta, p->zc, p->tw64x, p->tw64y, p->g.nx, p->g.ny, p->m, p->g.nz};
}

static ri_status forward_f64(ri_plan* p, const void* xv, void* bv, void* ws, size_t ws_bytes, void* stream) {
  const double* x = static_cast<const double*>(xv);
  double* b = static_cast<double*>(bv);
  const size_t vb = (size_t)p->g.nx * p->g.ny * p->g.nz * sizeof(double), hb = (size_t)p->g.nx * p->g.ny * sizeof(double);
  ri_status st = check_common(p, x, b, ws, ws_bytes, RI_OP_FORWARD, vb, hb);
  if (st != RI_OK) return st;
  if (overlaps(x, vb, b, hb)) return fail(RI_ERR_INVALID_ARG, "x and b_out overlap");
  const Layout64 L = layout64(p, RI_OP_FORWARD);
  HIP_TRY(forward64(tables64(p), x, b, at<double2>(ws, L.X), at<double2>(ws, L.S), (hipStream_t)stream));
  return RI_OK;
}

static ri_status adjoint_f64(ri_plan* p, const void* yv, void* xv, void* ws, size_t ws_bytes, void* stream) {
  const double* y = static_cast<const double*>(yv);
  double* x = static_cast<double*>(xv);
  const size_t vb = (size_t)p->g.nx * p->g.ny * p->g.nz * sizeof(double), hb = (size_t)p->g.nx * p->g.ny * sizeof(double);
  ri_status st = check_common(p, y, x, ws, ws_bytes, RI_OP_ADJOINT, hb, vb);
  if (st != RI_OK) return st;
  if (overlaps(y, hb, x, vb)) return fail(RI_ERR_INVALID_ARG, "y and x_out overlap");
  const Layout64 L = layout64(p, RI_OP_ADJOINT);
  HIP_TRY(adjoint64(tables64(p), y, x, at<double2>(ws, L.X), at<double2>(ws, L.S), (hipStream_t)stream));
  return RI_OK;
}

static Prox64Args prox64_args(const ri_plan* p, const Layout64& L, void* ws, int nonneg, int inner, double step,
                              double l1, double tv) {
  Prox64Args a{};
  const int parts = p->cplx ? 2 : 1;
  for (int k = 0; k < 3; ++k) {
    a.p[k] = L.p[k] ? at<double>(ws, L.p[k]) : nullptr;
    a.p2[k] = L.p2[k] ? at<double>(ws, L.p2[k]) : nullptr;
  }
  a.nx = p->g.nx;
  a.ny = p->g.ny;
  a.nz = p->g.nz / parts;
  a.parts = parts;
  a.tv2 = (p->g.flags & RI_TV2D) ? 1 : 0;
  a.nonneg = nonneg;
  a.inner_iters = inner;
  a.step = step;
  a.l1 = l1;
  a.tv = tv;
  return a;
}

static ri_status prox_f64(ri_plan* p, const ri_prox_params* pp, double step, const void* vv, void* xv, void* ws,
                          size_t ws_bytes, void* stream) {
  const double* v = static_cast<const double*>(vv);
  double* x = static_cast<double*>(xv);
  const size_t vb = (size_t)p->g.nx * p->g.ny * p->g.nz * sizeof(double);
  ri_status st = check_common(p, v, x, ws, ws_bytes, RI_OP_PROX, vb, vb);
  if (st != RI_OK) return st;
  if (v != x && overlaps(v, vb, x, vb)) return fail(RI_ERR_INVALID_ARG, "v and x_out partially overlap");
  if (!(step >= 0) || !std::isfinite(step) || !(pp->l1 >= 0) || !(pp->tv >= 0) || !std::isfinite(pp->l1) ||
      !std::isfinite(pp->tv) || pp->inner_iters < 0)
    return fail(RI_ERR_INVALID_ARG, "step, l1, tv must be finite and >= 0; inner_iters >= 0");
  Prox64Args a = prox64_args(p, layout64(p, RI_OP_PROX), ws, pp->nonneg ? 1 : 0, pp->inner_iters, step, pp->l1,
                             pp->tv);
  a.v = v;
  a.x = x;   // in place is allowed: the last launch reads only a voxel's own v
  HIP_TRY(launch_prox64(a, (hipStream_t)stream));
  return RI_OK;
}

// FISTA in FP64: x_k = prox(y_k - t A^T (A y_k - b)), s_{k+1} = (1 + sqrt(1 +
// 4 s_k^2)) / 2, y_{k+1} = x_k + ((s_k - 1)/s_{k+1}) (x_k - x_{k-1}), from
// x_0 = 0 or the given start (scaled).  The objective is evaluated (a forward
// model and the partials of sum |x| and TV) when a gap stop or the restart
// needs it, and for the returned iterate.
static ri_status solve_f64(ri_plan* p, const ri_solve_params* sp, const double* b, double* x, void* ws, hipStream_t s,
                           ri_solve_report* report) {
  const Layout64 L = layout64(p, RI_OP_SOLVE);
  const Plan64Tables t = tables64(p);
  const int parts = p->cplx ? 2 : 1;
  const int nzq = p->g.nz / parts;
  const int tv2 = (p->g.flags & RI_TV2D) ? 1 : 0;
  const size_t n = (size_t)p->g.nx * p->g.ny * p->g.nz, np = (size_t)p->g.nx * p->g.ny;
  double2* X = at<double2>(ws, L.X);
  double2* S = at<double2>(ws, L.S);
  double* hol = at<double>(ws, L.hol);
  double* y = at<double>(ws, L.y);
  double* xb = at<double>(ws, L.xp);
  double* v = at<double>(ws, L.v);
  double* part = at<double>(ws, L.part);
  double* psum = at<double>(ws, L.psum);
  double* ptv = at<double>(ws, L.ptv);
  const double tstep = 1.0 / p->lipschitz;
  Prox64Args pa = prox64_args(p, L, ws, sp->nonneg ? 1 : 0, sp->inner_iters, tstep, sp->l1, sp->tv);
  std::vector<double> h(3 * (size_t)L.nblk);
  auto objective = [&](const double* xv, double* F) -> hipError_t {
    hipError_t e = forward64(t, xv, hol, X, S, s);
    if (e == hipSuccess) e = sqdist64(hol, b, np, part, L.nblk, s);
    if (e == hipSuccess) e = launch_obj64(xv, p->g.nx, p->g.ny, nzq, parts, tv2, psum, ptv, L.nblk, s);
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), part, (size_t)L.nblk * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(h.data() + L.nblk, psum, (size_t)L.nblk * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(h.data() + 2 * L.nblk, ptv, (size_t)L.nblk * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    double d = 0.0, a1 = 0.0, a2 = 0.0;
    for (int i = 0; i < L.nblk; ++i) {
      d += h[i];
      a1 += h[L.nblk + i];
      a2 += h[2 * L.nblk + i];
    }
    *F = 0.5 * d + sp->l1 * a1 + sp->tv * a2;
    return hipSuccess;
  };
  // start
  if (sp->init == RI_INIT_ZERO) HIP_TRY(fill64(x, 0.0, n, s));
  else if (sp->x0_scale != 1.0) HIP_TRY(axpby64(x, sp->x0_scale, x, 0.0, x, n, s));
  HIP_TRY(hipMemcpyAsync(y, x, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  const bool restart = (sp->flags & RI_SOLVE_RESTART) != 0;
  const bool gap_stop = sp->f_ref > 0.0;
  const bool need_f = gap_stop || restart;
  double f0 = 0.0, f_prev = 0.0, f_cur = std::nan(""), f_min = INFINITY;
  int status = RI_OK, converged = 0, it = 0;
  auto judge = [&](double F) {   // after F(x_it): history, stop tests
    f_cur = F;
    f_min = std::min(f_min, F);
    if (!std::isfinite(F)) { status = RI_ERR_NONFINITE; return true; }
    if (it == 0) f0 = F;
    else if (F > 10.0 * f0 && F > 0.0) { status = RI_ERR_NOT_CONVERGED; return true; }
    if (gap_stop && (F - sp->f_ref) / sp->f_ref <= sp->gap_tol) { converged = 1; return true; }
    return false;
  };
  bool stop = false;
  if (need_f) {
    double F;
    HIP_TRY(objective(x, &F));
    stop = judge(F);
    f_prev = F;
  }
  double* xc = x;    // x_k
  double* xn = xb;   // x_{k+1} (held x_{k-1} until the prox writes it)
  double sk = 1.0;
  while (!stop && it < sp->max_iters) {
    HIP_TRY(forward64(t, y, hol, X, S, s));
    HIP_TRY(axpby64(hol, 1.0, hol, -1.0, b, np, s));          // r = A y - b
    HIP_TRY(adjoint64(t, hol, v, X, S, s));                   // A^T r
    HIP_TRY(axpby64(v, 1.0, y, -tstep, v, n, s));             // v = y - t A^T r
    pa.v = v;
    pa.x = xn;
    HIP_TRY(launch_prox64(pa, s));
    double s_new = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * sk * sk));
    double beta = (sk - 1.0) / s_new;
    ++it;
    if (need_f) {
      double F;
      HIP_TRY(objective(xn, &F));
      stop = judge(F);
      if (restart && F > f_prev) {
        s_new = 1.0;
        beta = 0.0;
      }
      f_prev = F;
    }
    HIP_TRY(axpby64(y, 1.0 + beta, xn, -beta, xc, n, s));    // y = x_new + beta (x_new - x)
    std::swap(xc, xn);
    sk = s_new;
  }
  if (xc != x) HIP_TRY(hipMemcpyAsync(x, xc, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (!report) {
    HIP_TRY(hipStreamSynchronize(s));
    return RI_OK;
  }
  if (!need_f || !std::isfinite(f_cur)) {
    double F;
    HIP_TRY(objective(x, &F));
    f_cur = F;
    f_min = std::min(f_min, F);
  }
  std::vector<double> hx(n);
  HIP_TRY(hipMemcpyAsync(hx.data(), x, n * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  size_t empty_rows = 0, empty_planes = 0;
  const int nrow = p->g.ny * p->g.nz;
  for (int r = 0; r < nrow; ++r) {
    bool any = false;
    for (int i = 0; i < p->g.nx && !any; ++i) any = hx[(size_t)r * p->g.nx + i] != 0.0;
    empty_rows += !any;
  }
  for (int z = 0; z < p->g.nz; ++z) {
    bool any = false;
    for (size_t i = 0; i < np && !any; ++i) any = hx[(size_t)z * np + i] != 0.0;
    empty_planes += !any;
  }
  std::memset(report, 0, sizeof(*report));
  report->iters = it;
  report->converged = converged;
  report->objective = f_cur;
  report->objective_min = f_min;
  report->gap = gap_stop ? (f_cur - sp->f_ref) / sp->f_ref : std::nan("");
  report->lipschitz = p->lipschitz;
  report->empty_row_frac = (double)empty_rows / (double)nrow;
  report->empty_plane_frac = (double)empty_planes / (double)p->g.nz;
  return (ri_status)status;
}

extern "C" ri_status ri_forward(ri_plan* p, const void* xv, void* bv, void* ws, size_t ws_bytes,
                                void* stream) {
  if (!p) return fail(RI_ERR_INVALID_ARG, "plan is NULL");
  if (p->dtype == RI_F64) return forward_f64(p, xv, bv, ws, ws_bytes, stream);
  const float* x = static_cast<const float*>(xv);
  float* b_out = static_cast<float*>(bv);
  const size_t vb = (size_t)p->g.nx * p->g.ny * p->g.nz * sizeof(float), hb = (size_t)p->g.nx * p->g.ny * sizeof(float);
  ri_status st = check_common(p, x, b_out, ws, ws_bytes, RI_OP_FORWARD, vb, hb);
  if (st != RI_OK) return st;
  if (overlaps(x, vb, b_out, hb)) return fail(RI_ERR_INVALID_ARG, "x and b_out overlap");
  HIP_TRY(enqueue_forward(p, make_layout(p, RI_OP_FORWARD), ws, x, b_out, (hipStream_t)stream));
  return RI_OK;
}

// ---------------------------------------------------------------------------
// Forward model without a caller workspace, for callers that cannot allocate
// (graph capture, serving loops).  Its scratch (the plane spectra, the
// z-chunk partial spectra and the summed hologram spectrum of ri_forward) lives
// in a fixed device array; every device the library runs on holds its own copy
// until the process ends.  Calls on one device share that copy, so calls that
// overlap on one device race; nothing in it needs clearing, since the forward
// writes every scratch element it later reads.
// ---------------------------------------------------------------------------
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device `dev` (current), looked up once per
// device.  The array's name is only a host-side handle for the symbol.
static ri_status static_scratch(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(RI_ERR_INVALID_ARG, "device %d outside 0..%d", dev, kMaxDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr)
      return fail(RI_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return RI_OK;
}

extern "C" size_t ri_forward_noalloc_max_scratch(void) { return kStaticScratchBytes; }

extern "C" ri_status ri_forward_noalloc(ri_plan* p, const void* xv, void* bv, void* stream) {
  if (!p) return fail(RI_ERR_INVALID_ARG, "plan is NULL");
  if (p->dtype == RI_F64) return fail(RI_ERR_INVALID_ARG, "ri_forward_noalloc takes RI_F32 plans only");
  const float* x = static_cast<const float*>(xv);
  float* b_out = static_cast<float*>(bv);
  if (!x || !b_out) return fail(RI_ERR_INVALID_ARG, "input or output pointer is NULL");
  if (((uintptr_t)x & 7) || ((uintptr_t)b_out & 7))
    return fail(RI_ERR_INVALID_ARG, "input and output must be 8-byte aligned");
  const size_t vb = (size_t)p->g.nx * p->g.ny * p->g.nz * sizeof(float), hb = (size_t)p->g.nx * p->g.ny * sizeof(float);
  if (overlaps(x, vb, b_out, hb)) return fail(RI_ERR_INVALID_ARG, "x and b_out overlap");
  const Layout L = make_layout(p, RI_OP_FORWARD);
  if (L.total > kStaticScratchBytes)
    return fail(RI_ERR_UNSUPPORTED_SIZE,
                "nx=%d ny=%d nz=%d needs %zu bytes of scratch; the allocation-free forward holds %zu "
                "(use ri_forward with a workspace)",
                p->g.nx, p->g.ny, p->g.nz, L.total, kStaticScratchBytes);
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != p->device) return fail(RI_ERR_INVALID_ARG, "plan belongs to device %d, current device is %d", p->device, dev);
  void* ws = nullptr;
  const ri_status st = static_scratch(dev, &ws);
  if (st != RI_OK) return st;
  if (overlaps(ws, kStaticScratchBytes, x, vb) || overlaps(ws, kStaticScratchBytes, b_out, hb))
    return fail(RI_ERR_INVALID_ARG, "an argument lies inside the library's scratch array");
  HIP_TRY(enqueue_forward(p, L, ws, x, b_out, (hipStream_t)stream));
  return RI_OK;
}

static hipError_t enqueue_adjoint(ri_plan* p, const Layout& L, void* ws, const float* y, float* x_out,
                                  hipStream_t s) {
  const PlanTables pt = p->tables();
  const int ny = p->g.ny, nz = p->g.nz, m = p->m;
  RowsR2CArgs ra{};
  ra.x = y;
  ra.out = at<float2>(ws, L.th);
  ra.nrows = ny;
  ra.mode = 0;
  ra.pt = pt;
  hipError_t e = launch_rows_r2c(m, ra, s);
  if (e != hipSuccess) return e;
  AdjColsArgs aa{};
  aa.th = at<float2>(ws, L.th);
  aa.u = at<float2>(ws, L.spec);
  aa.m = m;
  aa.nz = nz;
  aa.planes_per_chunk = L.ppc;
  aa.pt = pt;
  e = launch_adj_cols(ny, L.nchunk, aa, s);
  if (e != hipSuccess) return e;
  AdjRowsArgs ar{};
  ar.u = at<float2>(ws, L.spec);
  ar.nrows = ny * nz;
  ar.ny = ny;
  ar.out = x_out;
  ar.mode = 0;
  ar.scale = (float)(1.0 / ((double)p->g.nx * ny));
  ar.pt = pt;
  return launch_adj_rows(m, ar, s);
}

extern "C" ri_status ri_adjoint(ri_plan* p, const void* yv, void* xv, void* ws, size_t ws_bytes, void* stream) {
  if (!p) return fail(RI_ERR_INVALID_ARG, "plan is NULL");
  if (p->dtype == RI_F64) return adjoint_f64(p, yv, xv, ws, ws_bytes, stream);
  const float* y = static_cast<const float*>(yv);
  float* x_out = static_cast<float*>(xv);
  const size_t vb = (size_t)p->g.nx * p->g.ny * p->g.nz * sizeof(float), hb = (size_t)p->g.nx * p->g.ny * sizeof(float);
  ri_status st = check_common(p, y, x_out, ws, ws_bytes, RI_OP_ADJOINT, hb, vb);
  if (st != RI_OK) return st;
  if (overlaps(y, hb, x_out, vb)) return fail(RI_ERR_INVALID_ARG, "y and x_out overlap");
  HIP_TRY(enqueue_adjoint(p, make_layout(p, RI_OP_ADJOINT), ws, y, x_out, (hipStream_t)stream));
  return RI_OK;
}

extern "C" ri_status ri_prox_fused_lasso(ri_plan* p, const ri_prox_params* pp, double step, const void* vv,
                                         void* xv, void* ws, size_t ws_bytes, void* stream) {
  if (!p) return fail(RI_ERR_INVALID_ARG, "plan is NULL");
  const float* v = static_cast<const float*>(vv);
  float* x_out = static_cast<float*>(xv);
  if (!pp) return fail(RI_ERR_INVALID_ARG, "params is NULL");
  if (p->cplx && pp->nonneg) return fail(RI_ERR_INVALID_ARG, "nonneg has no meaning for a complex object (pass 0)");
  if (p->dtype == RI_F64) return prox_f64(p, pp, step, vv, xv, ws, ws_bytes, stream);
  const size_t vb = (size_t)p->g.nx * p->g.ny * p->g.nz * sizeof(float);
  ri_status st = check_common(p, v, x_out, ws, ws_bytes, RI_OP_PROX, vb, vb);
  if (st != RI_OK) return st;
  if (v != x_out && overlaps(v, vb, x_out, vb)) return fail(RI_ERR_INVALID_ARG, "v and x_out partially overlap");
  if (!(step >= 0) || !std::isfinite(step) || !(pp->l1 >= 0) || !(pp->tv >= 0) || !std::isfinite(pp->l1) ||
      !std::isfinite(pp->tv) || pp->inner_iters < 0)
    return fail(RI_ERR_INVALID_ARG, "step, l1, tv must be finite and >= 0; inner_iters >= 0");
  const Layout L = make_layout(p, RI_OP_PROX);
  ProxArgs a{};
  a.v = v;
  a.x = x_out;
  prox_duals(p, L, ws, &a);
  a.nx = p->g.nx;
  a.ny = p->g.ny;
  a.nz = p->g.nz;
  a.inner_iters = pp->inner_iters;
  a.nonneg = pp->nonneg ? 1 : 0;
  a.step = step;
  a.l1 = pp->l1;
  a.tv = pp->tv;
  a.levels = p->tune.tv_levels;
  a.blocks = p->tune.tv_blocks;
  // In place with TV active: the final pass reads v in each tile's halo and in
  // the z-margin of the neighbouring chunk while other blocks store x, and not
  // every block is resident at once, so x may not go into v's buffer.  The
  // final pass writes its result into the dual set it does not use (its
  // output set: it stores no dual) -- or, with bfloat16 duals, too small for
  // x, into a staging volume -- which is then copied over v.
  if (p->cplx) {   // in place is safe: the final launch reads only a voxel's own v
    HIP_TRY(launch_cprox(a, (hipStream_t)stream, nullptr));
    return RI_OK;
  }
  const double tau = step * pp->tv;
  const int K = (tau > 0.0 && pp->inner_iters > 0) ? pp->inner_iters : 0;
  float* staged = nullptr;
  if (v == x_out && K > 0) {
    const int npass = prox_passes(K, tau, p->tune.tv_levels, a.fgp != 0);
    if (plane_group(p) && !a.dual_bf16) {
      // the free dual set holds one group: each group's x is copied over v in turn
      a.stage_group = ((npass - 1) & 1) ? a.pa[0] : a.pb[0];
    } else {
      staged = a.dual_bf16 ? at<float>(ws, L.stage) : (((npass - 1) & 1) ? a.pa[0] : a.pb[0]);
      a.x = staged;
    }
  }
  HIP_TRY(launch_prox(a, (hipStream_t)stream, nullptr));
  if (staged != nullptr)
    HIP_TRY(launch_copy_f32(x_out, staged, (size_t)p->g.nx * p->g.ny * p->g.nz, (hipStream_t)stream));
  return RI_OK;
}

// ---------------------------------------------------------------------------
// Solve
// ---------------------------------------------------------------------------
enum { PH_FORWARD = 0, PH_HOLO = 1, PH_ADJOINT = 2, PH_PROX = 3, PH_OBJ = 4, PH_OTHER = 5 };

struct SolveCtx {
  ri_plan* p;
  Layout L;
  void* ws;
  const float* b;
  float* vol[3];
  SolveState* st;
  double step;
  double l1, tv;
  int inner;
  bool dense;
  int nonneg;
  bool warm;     // the TV dual carries over from one outer iteration to the next
  RowStores rs;  // row-compressed iterates (rs.on) or none
};

static RowStores row_stores(const ri_plan* p, const Layout& L, void* ws, float* x_inout) {
  RowStores rs{};
  if (L.cap == 0) return rs;
  for (int k = 0; k < 2; ++k) {
    rs.pool[k] = at<float>(ws, L.pool[k]);
    rs.slot[k] = at<int32_t>(ws, L.slot[k]);
  }
  rs.count = at<uint32_t>(ws, L.count);
  rs.overflow = at<uint32_t>(ws, L.overflow);
  rs.cap = L.cap;
  rs.nx = p->g.nx;
  rs.v = x_inout;
  rs.on = 1;
  return rs;
}

struct PhaseTimer {
  bool on = false;
  hipStream_t s = nullptr;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev;
  int launches[RI_NUM_PHASES] = {0};
  hipEvent_t open_ev = nullptr;
  int open_phase = -1;
  void begin(int ph) {
    if (!on) return;
    hipEventCreate(&open_ev);
    hipEventRecord(open_ev, s);
    open_phase = ph;
  }
  void end(int nlaunch) {
    if (!on) return;
    hipEvent_t e;
    hipEventCreate(&e);
    hipEventRecord(e, s);
    ev.push_back({open_phase, {open_ev, e}});
    launches[open_phase] += nlaunch;
  }
  void collect(double* ms, int* n) {
    for (auto& x : ev) {
      float t = 0.f;
      hipEventElapsedTime(&t, x.second.first, x.second.second);
      ms[x.first] += t;
      hipEventDestroy(x.second.first);
      hipEventDestroy(x.second.second);
    }
    for (int k = 0; k < RI_NUM_PHASES; ++k) n[k] += launches[k];
    ev.clear();
  }
};

// Argument structs of the kernels of one outer iteration of one frame.  The
// single-frame path launches them directly; the batched path uploads them.
struct IterArgs {
  ObjArgs obj;
  RowsR2CArgs fwd_rows;
  FwdColsArgs fwd_cols;
  HoloColsInvArgs holo_inv;
  RowsC2RArgs holo_c2r;
  ScalarArgs scal;
  RowsR2CArgs resid;
  AdjColsArgs adj_cols;
  AdjRowsArgs adj_rows;
  ProxArgs prox;
};

static IterArgs iteration_args(const SolveCtx& c) {
  ri_plan* p = c.p;
  const Layout& L = c.L;
  const PlanTables pt = p->tables();
  const int nx = p->g.nx, ny = p->g.ny, nz = p->g.nz, m = p->m;
  const float scale = (float)(1.0 / ((double)nx * ny));
  uint8_t* rowflag = at<uint8_t>(c.ws, L.rowflag);
  uint8_t* planeflag = at<uint8_t>(c.ws, L.planeflag);
  IterArgs I{};
  // objective pieces of x_it
  ObjArgs& oa = I.obj;
  oa.x0 = c.vol[0]; oa.x1 = c.vol[1]; oa.x2 = c.vol[2];
  oa.nx = nx; oa.ny = ny; oa.nz = nz;
  oa.rowflag = rowflag;
  oa.psum = at<double>(c.ws, L.psum);
  oa.ptv = at<double>(c.ws, L.ptv);
  oa.first_only = 1;
  oa.tv2 = (p->g.flags & RI_TV2D) ? 1 : 0;
  oa.rs = c.rs;
  oa.st = c.st;
  // A x_it (skipping empty rows and planes unless dense)
  RowsR2CArgs& ra = I.fwd_rows;
  for (int k = 0; k < 3; ++k) ra.xs[k] = c.vol[k];
  ra.out = at<float2>(c.ws, L.spec);
  ra.nrows = ny * nz;
  ra.rowflag = c.dense ? nullptr : rowflag;
  ra.st = c.st;
  ra.mode = 2;
  ra.rs = c.rs;
  ra.pt = pt;
  FwdColsArgs& fa = I.fwd_cols;
  fa.t = at<float2>(c.ws, L.spec);
  fa.gp = at<float2>(c.ws, L.gp);
  fa.m = m; fa.nz = nz; fa.planes_per_chunk = L.ppc;
  fa.rowflag = c.dense ? nullptr : rowflag;
  fa.planeflag = c.dense ? nullptr : planeflag;
  fa.st = c.st;
  fa.pt = pt;
  // hologram space: A x_it, data misfit, scalars, residual spectrum
  HoloColsInvArgs& ha = I.holo_inv;
  ha.gp = at<float2>(c.ws, L.gp);
  ha.gi = at<float2>(c.ws, L.gi);
  ha.m = m;
  ha.nchunk = L.nchunk;
  ha.st = c.st;
  ha.pt = pt;
  RowsC2RArgs& ca = I.holo_c2r;
  ca.in = at<float2>(c.ws, L.gi);
  ca.nrows = ny;
  ca.ax0 = at<float>(c.ws, L.ax0);
  ca.ax1 = at<float>(c.ws, L.ax1);
  ca.b = c.b;
  ca.partial = at<double>(c.ws, L.pdfit);
  ca.st = c.st;
  ca.mode = 1;
  ca.scale = scale;
  ca.pt = pt;
  ScalarArgs& sa = I.scal;
  sa.st = c.st;
  sa.pdfit = at<double>(c.ws, L.pdfit);
  sa.n_dfit = L.n_dfit;
  sa.psum = at<double>(c.ws, L.psum);
  sa.ptv = at<double>(c.ws, L.ptv);
  sa.n_obj = L.n_obj;
  sa.qsum = at<double>(c.ws, L.qsum);
  sa.qtv = at<double>(c.ws, L.qtv);
  sa.n_prox = plane_group(p) ? tv_group_final_blocks(nx, ny, nz, p->dual_planes, p->tune.tv_levels,
                                                      p->tune.tv_blocks, p->cus)
                             : tv_final_blocks(nx, ny, nz, p->tune.tv_levels, p->tune.tv_blocks, p->cus);
  sa.hist = at<double>(c.ws, L.hist);
  if (p->cplx) sa.qsum = sa.qtv = nullptr;   // the objective kernel runs every iteration
  sa.overflow = c.rs.on ? c.rs.overflow : nullptr;
  sa.count = c.rs.on ? c.rs.count : nullptr;
  RowsR2CArgs& rr = I.resid;
  rr.ax0 = at<float>(c.ws, L.ax0);
  rr.ax1 = at<float>(c.ws, L.ax1);
  rr.b = c.b;
  rr.out = at<float2>(c.ws, L.th);
  rr.nrows = ny;
  rr.st = c.st;
  rr.mode = 1;
  rr.pt = pt;
  // adjoint and gradient step: v = y - t A^T r over x_{it-1}
  AdjColsArgs& aa = I.adj_cols;
  aa.th = at<float2>(c.ws, L.th);
  aa.u = at<float2>(c.ws, L.spec);
  aa.m = m;
  aa.nz = nz;
  aa.planes_per_chunk = L.ppc;
  aa.st = c.st;
  aa.pt = pt;
  AdjRowsArgs& ar = I.adj_rows;
  ar.u = at<float2>(c.ws, L.spec);
  ar.nrows = ny * nz;
  ar.ny = ny;
  ar.x0 = c.vol[0]; ar.x1 = c.vol[1]; ar.x2 = c.vol[2];
  ar.rowflag = rowflag;
  ar.rowflag_prev = c.dense ? nullptr : at<uint8_t>(c.ws, L.rowflag_prev);
  ar.planeflag = planeflag;
  ar.st = c.st;
  ar.step = c.step;
  ar.mode = 1;
  ar.scale = scale;
  ar.rs = c.rs;
  ar.pt = pt;
  // fused-lasso prox -> x_{it+1}, occupancy flags
  ProxArgs& pa = I.prox;
  for (int k = 0; k < 3; ++k) pa.vol[k] = c.vol[k];
  prox_duals(p, L, c.ws, &pa);
  pa.rowflag = rowflag;
  pa.planeflag = planeflag;
  pa.psum = at<double>(c.ws, L.qsum);
  pa.ptv = at<double>(c.ws, L.qtv);
  pa.nx = nx; pa.ny = ny; pa.nz = nz;
  pa.inner_iters = c.inner;
  pa.nonneg = c.nonneg;
  pa.step = c.step;
  pa.l1 = c.l1;
  pa.tv = c.tv;
  pa.st = c.st;
  pa.levels = p->tune.tv_levels;
  pa.warm = c.warm ? 1 : 0;
  pa.blocks = p->tune.tv_blocks;
  pa.rs = c.rs;
  if (c.rs.on) pa.v = c.rs.v;   // v is the dense gradient-step output; x_{k+1} goes to a row store
  return I;
}

// One outer iteration: objective of x_it, momentum, gradient step, prox.
static hipError_t enqueue_iteration(const SolveCtx& c, hipStream_t s, PhaseTimer* tm) {
  const ri_plan* p = c.p;
  const int ny = p->g.ny, m = p->m;
  const IterArgs I = iteration_args(c);
  hipError_t e;
#define LTRY(x)                      \
  do {                               \
    e = (x);                         \
    if (e != hipSuccess) return e;   \
  } while (0)
  if (tm) tm->begin(PH_OBJ);
  LTRY(p->cplx ? launch_cobj(I.obj, c.L.n_obj, s) : launch_obj(I.obj, s));
  if (tm) tm->end(1);
  if (tm) tm->begin(PH_FORWARD);
  LTRY(launch_rows_r2c(m, I.fwd_rows, s));
  LTRY(launch_fwd_cols(ny, c.L.nchunk, I.fwd_cols, s));
  if (tm) tm->end(2);
  if (tm) tm->begin(PH_HOLO);
  LTRY(launch_holo_cols_inv(ny, I.holo_inv, s));
  LTRY(launch_rows_c2r(m, I.holo_c2r, s));
  LTRY(launch_scalars(I.scal, s));
  LTRY(launch_rows_r2c(m, I.resid, s));
  if (tm) tm->end(4);
  if (tm) tm->begin(PH_ADJOINT);
  LTRY(launch_adj_cols(ny, c.L.nchunk, I.adj_cols, s));
  LTRY(launch_adj_rows(m, I.adj_rows, s));
  if (tm) tm->end(2);
  if (tm) tm->begin(PH_PROX);
  int nl = 0;
  if (c.rs.on) LTRY(launch_store_clear_next(c.rs, ny, p->g.nz, c.st, s));
  LTRY(p->cplx ? launch_cprox(I.prox, s, &nl) : launch_prox(I.prox, s, &nl));
  if (tm) tm->end(nl);
#undef LTRY
  return hipSuccess;
}

static ri_status validate_solve(ri_plan* p, const ri_solve_params* sp, const float* b, float* x, void* ws,
                                size_t ws_bytes) {
  if (!p) return fail(RI_ERR_INVALID_ARG, "plan is NULL");
  if (!sp) return fail(RI_ERR_INVALID_ARG, "params is NULL");
  const size_t es = elem_bytes(p);
  const size_t vb = (size_t)p->g.nx * p->g.ny * p->g.nz * es, hb = (size_t)p->g.nx * p->g.ny * es;
  ri_status st = check_common(p, b, x, ws, ws_bytes, RI_OP_SOLVE, hb, vb);
  if (st != RI_OK) return st;
  if (overlaps(b, hb, x, vb)) return fail(RI_ERR_INVALID_ARG, "b and x_inout overlap");
  if (p->dtype == RI_F64 && (sp->flags & RI_SOLVE_DUAL_WARM))
    return fail(RI_ERR_INVALID_ARG, "RI_SOLVE_DUAL_WARM is not available with RI_F64 plans");
  if (!(sp->l1 >= 0) || !(sp->tv >= 0) || !std::isfinite(sp->l1) || !std::isfinite(sp->tv))
    return fail(RI_ERR_INVALID_ARG, "l1 and tv must be finite and >= 0");
  if (sp->max_iters < 0 || sp->inner_iters < 0) return fail(RI_ERR_INVALID_ARG, "iteration counts must be >= 0");
  if (sp->init != RI_INIT_ZERO && sp->init != RI_INIT_GIVEN) return fail(RI_ERR_INVALID_ARG, "init must be ZERO or GIVEN");
  if (!(sp->x0_scale >= 0) || !std::isfinite(sp->x0_scale))
    return fail(RI_ERR_INVALID_ARG, "x0_scale must be finite and >= 0");
  if (sp->f_ref > 0 && !(sp->gap_tol >= 0)) return fail(RI_ERR_INVALID_ARG, "gap_tol must be >= 0");
  if (sp->flags & ~(RI_SOLVE_DENSE | RI_SOLVE_NO_GRAPH | RI_SOLVE_RESTART | RI_SOLVE_TIMING | RI_SOLVE_DUAL_WARM |
                    RI_SOLVE_GROUPED))
    return fail(RI_ERR_INVALID_ARG, "unknown solve flags 0x%x", sp->flags);
  if ((sp->flags & RI_SOLVE_DUAL_WARM) && (p->g.flags & RI_TV_FGP))
    return fail(RI_ERR_INVALID_ARG, "RI_SOLVE_DUAL_WARM is not available with RI_TV_FGP plans");
  if (p->store_frac > 0.0 && (p->g.flags & RI_TV_DUAL_BF16))
    return fail(RI_ERR_INVALID_ARG, "row-compressed iterates are not available with RI_TV_DUAL_BF16 plans");
  if (p->cplx && sp->nonneg) return fail(RI_ERR_INVALID_ARG, "nonneg has no meaning for a complex object (pass 0)");
  if (p->cplx && (sp->flags & RI_SOLVE_DUAL_WARM))
    return fail(RI_ERR_INVALID_ARG, "RI_SOLVE_DUAL_WARM is not available with RI_COMPLEX plans");
  if (p->cplx && p->store_frac > 0.0)
    return fail(RI_ERR_INVALID_ARG, "row-compressed iterates are not available with RI_COMPLEX plans");
  if (plane_group(p) && (sp->flags & RI_SOLVE_DUAL_WARM))
    return fail(RI_ERR_INVALID_ARG, "RI_SOLVE_DUAL_WARM needs the whole dual (ri_plan_set_dual_planes 0)");
  if (plane_group(p) && p->store_frac > 0.0)
    return fail(RI_ERR_INVALID_ARG, "row-compressed iterates are not available with a plane-group dual");
  return RI_OK;
}

// Enqueue the solve set-up: state, x_0, x_{-1} = x_0, hologram buffers, flags.
static hipError_t enqueue_setup(const SolveCtx& c, const ri_solve_params* sp, hipStream_t s) {
  const ri_plan* p = c.p;
  const size_t nvox = (size_t)p->g.nx * p->g.ny * p->g.nz;
  const size_t npix = (size_t)p->g.nx * p->g.ny;
  StateInit in{};
  in.f_ref = sp->f_ref;
  in.gap_tol = sp->gap_tol;
  in.l1 = sp->l1;
  in.tv = sp->tv;
  in.max_iters = sp->max_iters;
  in.restart = (sp->flags & RI_SOLVE_RESTART) ? 1 : 0;
  hipError_t e = launch_state_init(c.st, in, s);
  if (e != hipSuccess) return e;
  uint8_t* rowflag = at<uint8_t>(c.ws, c.L.rowflag);
  uint8_t* planeflag = at<uint8_t>(c.ws, c.L.planeflag);
  if ((e = launch_fill_u8(rowflag, (size_t)p->g.ny * p->g.nz, 0, s)) != hipSuccess) return e;
  if ((e = launch_fill_u8(planeflag, (size_t)p->g.nz, 0, s)) != hipSuccess) return e;
  // x_{-1} is the start itself; its row flags are not known yet: every row may be occupied
  if ((e = launch_fill_u8(at<uint8_t>(c.ws, c.L.rowflag_prev), (size_t)p->g.ny * p->g.nz, 1, s)) != hipSuccess)
    return e;
  if (sp->init == RI_INIT_ZERO) {
    if (!c.rs.on && (e = launch_fill_f32(c.vol[0], nvox, 0.f, s)) != hipSuccess) return e;
  } else {
    if (sp->x0_scale != 0.0 && sp->x0_scale != 1.0)
      if ((e = launch_scale_f32(c.vol[0], nvox, (float)sp->x0_scale, s)) != hipSuccess) return e;
    if ((e = launch_flags_from_x(c.vol[0], p->g.nx, p->g.ny, p->g.nz, rowflag, planeflag, s)) != hipSuccess) return e;
  }
  if (c.rs.on) {
    // x_0 and x_{-1} into row stores 0 and 1 (all rows absent for a cold start)
    const float* x0 = sp->init == RI_INIT_ZERO ? nullptr : c.vol[0];
    if ((e = launch_store_start(c.rs, x0, p->g.ny, p->g.nz, s)) != hipSuccess) return e;
  } else {
    if ((e = launch_copy_f32(c.vol[2], c.vol[0], nvox, s)) != hipSuccess) return e;
  }
  if (c.warm) {
    // the first prox starts its dual from zero; it reads the first dual set
    const int nc = (p->g.flags & RI_TV2D) ? 2 : 3;
    const size_t nfill = (p->g.flags & RI_TV_DUAL_BF16) ? nvox / 2 : nvox;   // bf16 zeros are zero words
    for (int k = 0; k < nc; ++k)
      if ((e = launch_fill_f32(at<float>(c.ws, c.L.pa[k]), nfill, 0.f, s)) != hipSuccess) return e;
  }
  if ((e = launch_fill_f32(at<float>(c.ws, c.L.ax0), npix, 0.f, s)) != hipSuccess) return e;
  return launch_fill_f32(at<float>(c.ws, c.L.ax1), npix, 0.f, s);
}

// The final iterate into the caller's volume (from its row store, or from the
// rotating slot it ended in).
static hipError_t copy_out(const SolveCtx& c, float* x_out, hipStream_t s) {
  const ri_plan* p = c.p;
  if (c.rs.on) return launch_store_expand(c.rs, x_out, p->g.ny, p->g.nz, c.st, s);
  return launch_copy_final(c.vol[0], c.vol[1], c.vol[2], x_out, (size_t)p->g.nx * p->g.ny * p->g.nz, c.st, s);
}

static ri_status read_state(const SolveCtx& c, hipStream_t s, SolveState* out) {
  HIP_TRY(hipMemcpyAsync(out, c.st, sizeof(SolveState), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return RI_OK;
}

static ri_status get_graph(ri_plan* p, const SolveCtx& c, hipGraphExec_t* exec) {
  GraphCache& g = p->gc;
  if (g.exec && g.ws == c.ws && g.b == c.b && g.x == c.vol[0] && g.step == c.step && g.l1 == c.l1 &&
      g.tv == c.tv && g.inner == c.inner && g.dense == (int)c.dense && g.nonneg == c.nonneg &&
      g.warm == (int)c.warm && g.store_frac == c.p->store_frac) {
    *exec = g.exec;
    return RI_OK;
  }
  if (g.exec) { hipGraphExecDestroy(g.exec); g.exec = nullptr; }
  if (g.graph) { hipGraphDestroy(g.graph); g.graph = nullptr; }
  HIP_TRY(hipStreamBeginCapture(p->capture, hipStreamCaptureModeRelaxed));
  hipError_t e = enqueue_iteration(c, p->capture, nullptr);
  hipGraph_t graph = nullptr;
  hipError_t e2 = hipStreamEndCapture(p->capture, &graph);
  if (e != hipSuccess) { if (graph) hipGraphDestroy(graph); return fail(RI_ERR_HIP, "capture: %s", hipGetErrorString(e)); }
  if (e2 != hipSuccess) return fail(RI_ERR_HIP, "end capture: %s", hipGetErrorString(e2));
  hipGraphExec_t ex = nullptr;
  e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) { hipGraphDestroy(graph); return fail(RI_ERR_HIP, "instantiate: %s", hipGetErrorString(e)); }
  g.graph = graph;
  g.exec = ex;
  g.ws = c.ws; g.b = c.b; g.x = c.vol[0]; g.step = c.step; g.l1 = c.l1; g.tv = c.tv;
  g.inner = c.inner; g.dense = (int)c.dense; g.nonneg = c.nonneg; g.warm = (int)c.warm;
  g.store_frac = c.p->store_frac;
  *exec = ex;
  return RI_OK;
}

static ri_status fill_report(const SolveCtx& c, hipStream_t s, ri_solve_report* rep, PhaseTimer* tm) {
  SolveState h{};
  ri_status rs = read_state(c, s, &h);
  if (rs != RI_OK) return rs;
  const ri_plan* p = c.p;
  std::vector<uint8_t> rf((size_t)p->g.ny * p->g.nz), pf(p->g.nz);
  HIP_TRY(hipMemcpy(rf.data(), at<uint8_t>(c.ws, c.L.rowflag), rf.size(), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(pf.data(), at<uint8_t>(c.ws, c.L.planeflag), pf.size(), hipMemcpyDeviceToHost));
  size_t er = 0, ep = 0;
  for (auto v : rf) er += (v == 0);
  for (auto v : pf) ep += (v == 0);
  std::memset(rep, 0, sizeof(*rep));
  rep->iters = h.it;
  rep->converged = h.converged;
  rep->objective = h.f_cur;
  {
    const int nh = std::min(h.it + 1, kHistCap);
    std::vector<double> hist(nh);
    HIP_TRY(hipMemcpy(hist.data(), at<double>(c.ws, c.L.hist), nh * sizeof(double), hipMemcpyDeviceToHost));
    rep->objective_min = *std::min_element(hist.begin(), hist.end());
  }
  rep->gap = h.gap;
  rep->lipschitz = p->lipschitz;
  rep->empty_row_frac = (double)er / (double)rf.size();
  rep->empty_plane_frac = (double)ep / (double)pf.size();
  rep->store_rows_peak = h.rows_peak;
  if (tm) tm->collect(rep->phase_ms, rep->phase_launches);
  return (ri_status)h.status;
}

extern "C" ri_status ri_solve(ri_plan* p, const ri_solve_params* sp, const void* bv, void* xv, void* ws,
                              size_t ws_bytes, void* stream, ri_solve_report* report) {
  const float* b = static_cast<const float*>(bv);
  float* x_inout = static_cast<float*>(xv);
  ri_status vs = validate_solve(p, sp, b, x_inout, ws, ws_bytes);
  if (vs != RI_OK) return vs;
  if (p->dtype == RI_F64)
    return solve_f64(p, sp, static_cast<const double*>(bv), static_cast<double*>(xv), ws, (hipStream_t)stream, report);
  hipStream_t s = (hipStream_t)stream;
  SolveCtx c{};
  c.p = p;
  c.L = make_layout(p, RI_OP_SOLVE);
  c.ws = ws;
  c.b = b;
  c.vol[0] = x_inout;
  c.vol[1] = c.L.cap ? nullptr : at<float>(ws, c.L.vol1);
  c.vol[2] = c.L.cap ? nullptr : at<float>(ws, c.L.vol2);   // row stores replace slot 2
  c.rs = row_stores(p, c.L, ws, x_inout);
  c.st = at<SolveState>(ws, c.L.state);
  c.step = 1.0 / p->lipschitz;
  c.l1 = sp->l1;
  c.tv = sp->tv;
  c.inner = sp->inner_iters;
  c.dense = (sp->flags & RI_SOLVE_DENSE) != 0;
  c.nonneg = sp->nonneg ? 1 : 0;
  c.warm = (sp->flags & RI_SOLVE_DUAL_WARM) != 0;
  const bool timing = (sp->flags & RI_SOLVE_TIMING) != 0 && report != nullptr;
  const bool use_graph = !timing && !(sp->flags & RI_SOLVE_NO_GRAPH);
  PhaseTimer tm;
  tm.on = timing;
  tm.s = s;

  if (timing) tm.begin(PH_OTHER);
  HIP_TRY(enqueue_setup(c, sp, s));
  if (timing) tm.end(6);
  hipGraphExec_t exec = nullptr;
  if (use_graph) {
    ri_status gs = get_graph(p, c, &exec);
    if (gs != RI_OK) return gs;
  }
  const int total = sp->max_iters + 1;  // the last group only evaluates the final objective
  // with phase timing every launched group is counted, so poll after each one
  const int every = timing ? 1 : std::max(1, sp->check_every);
  const bool poll = sp->f_ref > 0;
  for (int k = 0; k < total; ++k) {
    if (use_graph) {
      HIP_TRY(hipGraphLaunch(exec, s));
    } else {
      HIP_TRY(enqueue_iteration(c, s, timing ? &tm : nullptr));
    }
    if (poll && ((k + 1) % every == 0) && k + 1 < total) {
      HIP_TRY(hipMemcpyAsync(p->host_flag, &c.st->done, sizeof(int32_t), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      if (*p->host_flag) break;
    }
  }
  if (timing) tm.begin(PH_OTHER);
  HIP_TRY(copy_out(c, x_inout, s));
  if (timing) tm.end(1);
  if (!report) return RI_OK;
  return fill_report(c, s, report, timing ? &tm : nullptr);
}

// ---------------------------------------------------------------------------
// Batched solve.  Frames advance in lock-step; every kernel of an iteration is
// launched once per transform size (rows: nx/2, columns: ny) or once for all
// frames (objective, scalars, TV passes), with per-frame argument structs and
// block offsets uploaded once into a table region at the end of the workspace.
// One iteration of all frames is captured as one HIP graph and replayed until
// a device-side count of stopped frames reaches n.
// ---------------------------------------------------------------------------
enum BatchKind { BK_OBJ, BK_FWD_ROWS, BK_FWD_COLS, BK_HOLO_INV, BK_HOLO_C2R, BK_SCAL, BK_RESID, BK_ADJ_COLS,
                 BK_ADJ_ROWS, BK_TV, BK_COUNT };

struct BatchLaunch {
  int kind;
  int size;       // template size (m or ny), 0 when the kernel is not specialised
  int pass;       // TV pass index
  bool final_pass = false;  // TV: the frames' final pass
  bool tv2 = false;         // TV: per-plane 2D TV frames
  bool fgp = false;         // TV: accelerated-dual frames
  bool bf16 = false;        // TV: bfloat16-dual frames
  bool sparse = false;      // TV: frames with row-compressed iterates
  std::vector<int> frames;
  size_t args_off = 0, offs_off = 0;
  size_t queue_off = 0;     // TV: claim counters of the persistent form
  int nblocks = 0;
};

static size_t kind_args_size(int kind) {
  switch (kind) {
    case BK_OBJ: return sizeof(ObjArgs);
    case BK_FWD_ROWS: case BK_RESID: return sizeof(RowsR2CArgs);
    case BK_FWD_COLS: return sizeof(FwdColsArgs);
    case BK_HOLO_INV: return sizeof(HoloColsInvArgs);
    case BK_HOLO_C2R: return sizeof(RowsC2RArgs);
    case BK_SCAL: return sizeof(ScalarArgs);
    case BK_ADJ_COLS: return sizeof(AdjColsArgs);
    case BK_ADJ_ROWS: return sizeof(AdjRowsArgs);
    case BK_TV: return tv_pass_args_size();
  }
  return 0;
}

static int prox_pass_count(const ri_plan* p, const ri_solve_params& sp) {
  return prox_passes(sp.inner_iters, (1.0 / p->lipschitz) * sp.tv, p->tune.tv_levels, (p->g.flags & RI_TV_FGP) != 0);
}

// The launches of one batched iteration (frames grouped by transform size).
static std::vector<BatchLaunch> batch_launches(int n, ri_plan* const* plans, const ri_solve_params* params) {
  std::vector<BatchLaunch> out;
  auto group = [&](int kind, bool by_m, bool by_ny) {
    std::vector<int> sizes;
    for (int i = 0; i < n; ++i) {
      const int key = by_m ? plans[i]->m : (by_ny ? plans[i]->g.ny : 0);
      if (std::find(sizes.begin(), sizes.end(), key) == sizes.end()) sizes.push_back(key);
    }
    for (int key : sizes) {
      BatchLaunch b;
      b.kind = kind;
      b.size = key;
      b.pass = 0;
      for (int i = 0; i < n; ++i) {
        const int k2 = by_m ? plans[i]->m : (by_ny ? plans[i]->g.ny : 0);
        if (k2 == key) b.frames.push_back(i);
      }
      out.push_back(b);
    }
  };
  group(BK_OBJ, false, false);
  group(BK_FWD_ROWS, true, false);
  group(BK_FWD_COLS, false, true);
  group(BK_HOLO_INV, false, true);
  group(BK_HOLO_C2R, true, false);
  group(BK_SCAL, false, false);
  group(BK_RESID, true, false);
  group(BK_ADJ_COLS, false, true);
  group(BK_ADJ_ROWS, true, false);
  // TV pass p of every frame that has one, one launch per fusion depth and
  // per kind of pass (a dual pass, or a frame's final pass)
  int maxpass = 0;
  for (int i = 0; i < n; ++i) maxpass = std::max(maxpass, prox_pass_count(plans[i], params[i]));
  for (int p = 0; p < maxpass; ++p) {
    for (int fin = 0; fin < 2; ++fin) {
      for (int t2 = 0; t2 < 2; ++t2) {
        for (int fg = 0; fg < 8; ++fg) {   // bit 0: FGP, bit 1: bfloat16 dual, bit 2: row stores
          for (int H = kTvLevelsMin; H <= kTvLevelsMax; ++H) {
            BatchLaunch b;
            b.kind = BK_TV;
            b.size = H;
            b.pass = p;
            b.final_pass = fin != 0;
            b.tv2 = t2 != 0;
            b.fgp = (fg & 1) != 0;
            b.bf16 = (fg & 2) != 0;
            b.sparse = (fg & 4) != 0;
            for (int i = 0; i < n; ++i) {
              const int np = prox_pass_count(plans[i], params[i]);
              const bool f2 = (plans[i]->g.flags & RI_TV2D) != 0;
              const bool ff = (plans[i]->g.flags & RI_TV_FGP) != 0;
              const bool fb = (plans[i]->g.flags & RI_TV_DUAL_BF16) != 0;
              const bool fs = (p == np - 1) && plans[i]->store_frac > 0.0;   // only the final pass writes a store
              if (prox_levels(plans[i]->tune.tv_levels, ff) == H && p < np && (p == np - 1) == (fin != 0) &&
                  f2 == (t2 != 0) && ff == b.fgp && fb == b.bf16 && fs == b.sparse)
                b.frames.push_back(i);
            }
            if (!b.frames.empty()) out.push_back(b);
          }
        }
      }
    }
  }
  return out;
}

static size_t batch_tables_bytes(int n, ri_plan* const* plans, const ri_solve_params* params) {
  size_t off = 0;
  for (const BatchLaunch& b : batch_launches(n, plans, params)) {
    off = align_up(off + kind_args_size(b.kind) * b.frames.size());
    off = align_up(off + sizeof(uint32_t) * (b.frames.size() + 1));
    if (b.kind == BK_TV) off = align_up(off + sizeof(uint32_t) * kQueueWords);
  }
  off = align_up(off + sizeof(SolveState*) * n);  // states for the stop count
  off = align_up(off + sizeof(int32_t));           // the count
  return off;
}

static size_t frame_ws_bytes(const ri_plan* p) { return align_up(make_layout(p, RI_OP_SOLVE).total); }

extern "C" ri_status ri_workspace_size_batched(int32_t n, ri_plan* const* plans, const ri_solve_params* params,
                                               size_t* bytes) {
  if (!bytes || n < 0 || (n > 0 && (!plans || !params))) return fail(RI_ERR_INVALID_ARG, "invalid argument");
  size_t tot = 256;
  for (int i = 0; i < n; ++i) {
    if (!plans[i]) return fail(RI_ERR_INVALID_ARG, "plans[%d] is NULL", i);
    tot += frame_ws_bytes(plans[i]);
  }
  *bytes = tot + batch_tables_bytes(n, plans, params);
  return RI_OK;
}

extern "C" ri_status ri_solve_batched(int32_t n, ri_plan* const* plans, const ri_solve_params* params,
                                      const void* const* bv, void* const* xv, void* ws, size_t ws_bytes,
                                      void* stream, ri_solve_report* reports) {
  const float* const* b = reinterpret_cast<const float* const*>(bv);
  float* const* x_inout = reinterpret_cast<float* const*>(xv);
  if (n < 0) return fail(RI_ERR_INVALID_ARG, "n < 0");
  if (n == 0) return RI_OK;
  if (!plans || !params || !b || !x_inout) return fail(RI_ERR_INVALID_ARG, "NULL array argument");
  size_t need = 0;
  ri_status vs = ri_workspace_size_batched(n, plans, params, &need);
  if (vs != RI_OK) return vs;
  if (!ws) return fail(RI_ERR_INVALID_ARG, "workspace is NULL");
  if (ws_bytes < need) return fail(RI_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes < %zu required", ws_bytes, need);
  hipStream_t s = (hipStream_t)stream;
  // frame workspaces from an aligned base, tables after them
  char* base = (char*)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
  std::vector<SolveCtx> ctx(n);
  size_t off = 0;
  for (int i = 0; i < n; ++i) {
    ri_plan* p = plans[i];
    const size_t fb = frame_ws_bytes(p);
    vs = validate_solve(p, &params[i], b[i], x_inout[i], base + off, fb);
    if (vs != RI_OK) return vs;
    if (p->cplx) return fail(RI_ERR_INVALID_ARG, "frame %d: RI_COMPLEX plans are solved one by one (ri_solve)", i);
    if (p->dtype == RI_F64) return fail(RI_ERR_INVALID_ARG, "frame %d: RI_F64 plans are solved one by one (ri_solve)", i);
    if (plane_group(p))
      return fail(RI_ERR_INVALID_ARG, "frame %d: plane-group duals are solved one by one (ri_solve)", i);
    if (p->device != plans[0]->device) return fail(RI_ERR_INVALID_ARG, "plans on different devices");
    SolveCtx& c = ctx[i];
    c.p = p;
    c.L = make_layout(p, RI_OP_SOLVE);
    c.ws = base + off;
    c.b = b[i];
    c.vol[0] = x_inout[i];
    c.vol[1] = c.L.cap ? nullptr : at<float>(c.ws, c.L.vol1);
    c.vol[2] = c.L.cap ? nullptr : at<float>(c.ws, c.L.vol2);
    c.rs = row_stores(plans[i], c.L, c.ws, x_inout[i]);
    c.st = at<SolveState>(c.ws, c.L.state);
    c.step = 1.0 / p->lipschitz;
    c.l1 = params[i].l1;
    c.tv = params[i].tv;
    c.inner = params[i].inner_iters;
    c.dense = (params[i].flags & RI_SOLVE_DENSE) != 0;
    c.nonneg = params[i].nonneg ? 1 : 0;
    c.warm = (params[i].flags & RI_SOLVE_DUAL_WARM) != 0;
    off += fb;
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      if (i != j && overlaps(x_inout[i], (size_t)plans[i]->g.nx * plans[i]->g.ny * plans[i]->g.nz * 4, x_inout[j],
                             (size_t)plans[j]->g.nx * plans[j]->g.ny * plans[j]->g.nz * 4))
        return fail(RI_ERR_INVALID_ARG, "x_inout[%d] and x_inout[%d] overlap", i, j);
  char* tables = base + off;

  // per-frame argument structs (grids filled in as the single-frame launchers do)
  std::vector<IterArgs> it(n);
  std::vector<std::vector<char>> tv(n);
  std::vector<std::vector<int>> tv_blocks(n);
  std::vector<int> npass(n);
  for (int i = 0; i < n; ++i) {
    it[i] = iteration_args(ctx[i]);
    const ri_plan* p = plans[i];
    const int ny = p->g.ny, nz = p->g.nz, m = p->m;
    dim3 g;
    g = grid_obj(p->g.nx, ny, nz);             it[i].obj.gx = g.x; it[i].obj.gy = g.y;
    g = grid_rows(m, ny * nz);                 it[i].fwd_rows.gx = g.x; it[i].fwd_rows.gy = g.y;
    g = grid_cols(ny, m, ctx[i].L.nchunk);     it[i].fwd_cols.gx = g.x; it[i].fwd_cols.gy = g.y;
    g = grid_cols(ny, m, 1);                   it[i].holo_inv.gx = g.x; it[i].holo_inv.gy = g.y;
    g = grid_rows(m, ny);                      it[i].holo_c2r.gx = g.x; it[i].holo_c2r.gy = g.y;
    it[i].scal.gx = 1; it[i].scal.gy = 1;
    g = grid_rows(m, ny);                      it[i].resid.gx = g.x; it[i].resid.gy = g.y;
    g = grid_cols(ny, m, ctx[i].L.nchunk);     it[i].adj_cols.gx = g.x; it[i].adj_cols.gy = g.y;
    g = grid_rows(m, ny * nz);                 it[i].adj_rows.gx = g.x; it[i].adj_rows.gy = g.y;
    npass[i] = prox_pass_count(p, params[i]);
    tv[i].resize(tv_pass_args_size() * npass[i]);
    tv_blocks[i].resize(npass[i]);
    prox_pass_args(it[i].prox, tv[i].data(), tv_blocks[i].data());
  }
  auto frame_blocks = [&](int kind, int pass, int i) -> int {
    const IterArgs& a = it[i];
    switch (kind) {
      case BK_OBJ: return a.obj.gx * a.obj.gy;
      case BK_FWD_ROWS: return a.fwd_rows.gx * a.fwd_rows.gy;
      case BK_FWD_COLS: return a.fwd_cols.gx * a.fwd_cols.gy;
      case BK_HOLO_INV: return a.holo_inv.gx * a.holo_inv.gy;
      case BK_HOLO_C2R: return a.holo_c2r.gx * a.holo_c2r.gy;
      case BK_SCAL: return 1;
      case BK_RESID: return a.resid.gx * a.resid.gy;
      case BK_ADJ_COLS: return a.adj_cols.gx * a.adj_cols.gy;
      case BK_ADJ_ROWS: return a.adj_rows.gx * a.adj_rows.gy;
      case BK_TV: return tv_blocks[i][pass];
    }
    return 0;
  };
  auto frame_args = [&](int kind, int pass, int i) -> const void* {
    const IterArgs& a = it[i];
    switch (kind) {
      case BK_OBJ: return &a.obj;
      case BK_FWD_ROWS: return &a.fwd_rows;
      case BK_FWD_COLS: return &a.fwd_cols;
      case BK_HOLO_INV: return &a.holo_inv;
      case BK_HOLO_C2R: return &a.holo_c2r;
      case BK_SCAL: return &a.scal;
      case BK_RESID: return &a.resid;
      case BK_ADJ_COLS: return &a.adj_cols;
      case BK_ADJ_ROWS: return &a.adj_rows;
      case BK_TV: return tv[i].data() + tv_pass_args_size() * pass;
    }
    return nullptr;
  };
  // stage the tables on the host, upload once
  std::vector<BatchLaunch> launches = batch_launches(n, plans, params);
  const size_t tbytes = batch_tables_bytes(n, plans, params);
  std::vector<char> host(tbytes, 0);
  size_t t = 0;
  for (BatchLaunch& bl : launches) {
    const size_t as = kind_args_size(bl.kind);
    bl.args_off = t;
    for (size_t k = 0; k < bl.frames.size(); ++k)
      std::memcpy(host.data() + t + k * as, frame_args(bl.kind, bl.pass, bl.frames[k]), as);
    t = align_up(t + as * bl.frames.size());
    bl.offs_off = t;
    uint32_t* o = reinterpret_cast<uint32_t*>(host.data() + t);
    uint32_t acc = 0;
    for (size_t k = 0; k < bl.frames.size(); ++k) {
      o[k] = acc;
      acc += (uint32_t)frame_blocks(bl.kind, bl.pass, bl.frames[k]);
    }
    o[bl.frames.size()] = acc;
    bl.nblocks = (int)acc;
    t = align_up(t + sizeof(uint32_t) * (bl.frames.size() + 1));
    if (bl.kind == BK_TV) {  // counters staged as zeros
      bl.queue_off = t;
      t = align_up(t + sizeof(uint32_t) * kQueueWords);
    }
  }
  const size_t states_off = t;
  for (int i = 0; i < n; ++i) reinterpret_cast<SolveState**>(host.data() + t)[i] = ctx[i].st;
  t = align_up(t + sizeof(SolveState*) * n);
  const size_t count_off = t;
  HIP_TRY(hipMemcpyAsync(tables, host.data(), tbytes, hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));  // the staging buffer is pageable and local

  const bool persistent = (params[0].flags & RI_SOLVE_GROUPED) == 0;
  auto enqueue_batch_iteration = [&](hipStream_t q) -> hipError_t {
    hipError_t e = hipSuccess;
    bool cleared = false;
    for (const BatchLaunch& bl : launches) {
      if (bl.nblocks == 0) continue;
      BatchMap mp{reinterpret_cast<const uint32_t*>(tables + bl.offs_off), (int)bl.frames.size()};
      if (persistent && bl.kind == BK_TV) {
        mp.queue = reinterpret_cast<uint32_t*>(tables + bl.queue_off);
        mp.grid = std::max(1, plans[0]->cus);
      }
      const void* a = tables + bl.args_off;
      switch (bl.kind) {
        case BK_OBJ: e = launch_obj_batched((const ObjArgs*)a, mp, bl.nblocks, q); break;
        case BK_FWD_ROWS: case BK_RESID:
          e = launch_rows_r2c_batched(bl.size, (const RowsR2CArgs*)a, mp, bl.nblocks, q); break;
        case BK_FWD_COLS: e = launch_fwd_cols_batched(bl.size, (const FwdColsArgs*)a, mp, bl.nblocks, q); break;
        case BK_HOLO_INV:
          e = launch_holo_cols_inv_batched(bl.size, (const HoloColsInvArgs*)a, mp, bl.nblocks, q); break;
        case BK_HOLO_C2R: e = launch_rows_c2r_batched(bl.size, (const RowsC2RArgs*)a, mp, bl.nblocks, q); break;
        case BK_SCAL: e = launch_scalars_batched((const ScalarArgs*)a, mp, bl.nblocks, q); break;
        case BK_ADJ_COLS: e = launch_adj_cols_batched(bl.size, (const AdjColsArgs*)a, mp, bl.nblocks, q); break;
        case BK_ADJ_ROWS: e = launch_adj_rows_batched(bl.size, (const AdjRowsArgs*)a, mp, bl.nblocks, q); break;
        case BK_TV:
          if (!cleared) {
            // the stores that this iteration's final passes fill start empty
            for (int i = 0; i < n && e == hipSuccess; ++i)
              if (ctx[i].rs.on) e = launch_store_clear_next(ctx[i].rs, plans[i]->g.ny, plans[i]->g.nz, ctx[i].st, q);
            cleared = true;
            if (e != hipSuccess) return e;
          }
          e = launch_tv_pass_batched(bl.size, bl.final_pass, bl.tv2, bl.fgp, bl.bf16, bl.sparse, a, mp, bl.nblocks,
                                     q);
          break;
      }
      if (e != hipSuccess) return e;
    }
    return launch_count_done(reinterpret_cast<SolveState* const*>(tables + states_off), n,
                             reinterpret_cast<int32_t*>(tables + count_off), q);
  };

  for (int i = 0; i < n; ++i) HIP_TRY(enqueue_setup(ctx[i], &params[i], s));
  const bool use_graph = !(params[0].flags & RI_SOLVE_NO_GRAPH);
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  if (use_graph) {
    hipStream_t cap = plans[0]->capture;
    HIP_TRY(hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed));
    hipError_t e = enqueue_batch_iteration(cap);
    hipError_t e2 = hipStreamEndCapture(cap, &graph);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (graph) hipGraphDestroy(graph);
      return fail(RI_ERR_HIP, "batch capture: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    }
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      hipGraphDestroy(graph);
      return fail(RI_ERR_HIP, "batch instantiate: %s", hipGetErrorString(e));
    }
  }
  int total = 0, every = 1 << 30;
  for (int i = 0; i < n; ++i) {
    total = std::max(total, params[i].max_iters + 1);
    every = std::min(every, std::max(1, params[i].check_every));
  }
  ri_status rs = RI_OK;
  for (int k = 0; k < total && rs == RI_OK; ++k) {
    hipError_t e = use_graph ? hipGraphLaunch(exec, s) : enqueue_batch_iteration(s);
    if (e != hipSuccess) rs = fail(RI_ERR_HIP, "batch iteration: %s", hipGetErrorString(e));
    if (rs == RI_OK && (k + 1) % every == 0 && k + 1 < total) {
      int32_t* hf = plans[0]->host_flag;
      e = hipMemcpyAsync(hf, tables + count_off, sizeof(int32_t), hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) rs = fail(RI_ERR_HIP, "batch poll: %s", hipGetErrorString(e));
      else if (*hf >= n) break;
    }
  }
  if (exec) hipGraphExecDestroy(exec);
  if (graph) hipGraphDestroy(graph);
  if (rs != RI_OK) return rs;
  for (int i = 0; i < n; ++i)
    HIP_TRY(copy_out(ctx[i], x_inout[i], s));
  if (!reports) return RI_OK;
  ri_status agg = RI_OK;
  for (int i = 0; i < n; ++i) {
    const ri_status st = fill_report(ctx[i], s, &reports[i], nullptr);
    if (st != RI_OK && agg == RI_OK) agg = st;
  }
  return agg;
}

// ---------------------------------------------------------------------------
// Tuning: launch shapes per geometry, chosen by timing on the device and kept
// in an optional cache file (one JSON object per line).
// ---------------------------------------------------------------------------
static ri_status validate_tuning(const ri_tuning* t) {
  if (!t) return fail(RI_ERR_INVALID_ARG, "tuning is NULL");
  if (t->tv_levels < kTvLevelsMin || t->tv_levels > kTvLevelsMax)
    return fail(RI_ERR_INVALID_ARG, "tv_levels=%d must be in [%d, %d]", t->tv_levels, kTvLevelsMin, kTvLevelsMax);
  if (t->tv_blocks < 64 || t->tv_blocks > 65536)
    return fail(RI_ERR_INVALID_ARG, "tv_blocks=%d must be in [64, 65536]", t->tv_blocks);
  if (t->col_blocks < kColMinBlocks || t->col_blocks > kColMaxBlocks)
    return fail(RI_ERR_INVALID_ARG, "col_blocks=%d must be in [%d, %d]", t->col_blocks, kColMinBlocks, kColMaxBlocks);
  return RI_OK;
}

extern "C" ri_status ri_plan_get_tuning(const ri_plan* p, ri_tuning* out) {
  if (!p || !out) return fail(RI_ERR_INVALID_ARG, "NULL argument");
  *out = p->tune;
  return RI_OK;
}

extern "C" ri_status ri_plan_set_tuning(ri_plan* p, const ri_tuning* t) {
  if (!p) return fail(RI_ERR_INVALID_ARG, "plan is NULL");
  const ri_status vs = validate_tuning(t);
  if (vs != RI_OK) return vs;
  p->tune = *t;
  drop_graph(p);
  return RI_OK;
}

extern "C" ri_status ri_plan_set_storage(ri_plan* p, double row_fraction) {
  if (!p) return fail(RI_ERR_INVALID_ARG, "plan is NULL");
  if (!(row_fraction >= 0.0 && row_fraction <= 1.0))
    return fail(RI_ERR_INVALID_ARG, "row_fraction=%g must be in [0, 1]", row_fraction);
  if (row_fraction > 0.0 && p->dtype == RI_F64)
    return fail(RI_ERR_INVALID_ARG, "row-compressed iterates are not available with RI_F64 plans");
  p->store_frac = row_fraction;
  drop_graph(p);
  return RI_OK;
}

extern "C" ri_status ri_plan_set_dual_planes(ri_plan* p, int32_t planes) {
  if (!p) return fail(RI_ERR_INVALID_ARG, "plan is NULL");
  if (planes < 0) return fail(RI_ERR_INVALID_ARG, "planes=%d must be >= 0", planes);
  if (planes > 0 && !(p->g.flags & RI_TV2D))
    return fail(RI_ERR_INVALID_ARG, "a dual of a few planes needs the per-plane 2D TV (RI_TV2D)");
  if (planes > 0 && (p->cplx || p->dtype == RI_F64 || (p->g.flags & RI_TV_FGP)))
    return fail(RI_ERR_INVALID_ARG, "plane-group duals are for RI_F32 real plans without RI_TV_FGP");
  p->dual_planes = planes;
  drop_graph(p);
  return RI_OK;
}

extern "C" ri_status ri_plan_get_dual_planes(const ri_plan* p, int32_t* planes) {
  if (!p || !planes) return fail(RI_ERR_INVALID_ARG, "NULL argument");
  *planes = p->dual_planes;
  return RI_OK;
}

extern "C" ri_status ri_plan_get_storage(const ri_plan* p, double* row_fraction) {
  if (!p || !row_fraction) return fail(RI_ERR_INVALID_ARG, "NULL argument");
  *row_fraction = p->store_frac;
  return RI_OK;
}

static std::string tune_key(const ri_plan* p, int inner) {
  hipDeviceProp_t prop{};
  char arch[96] = "unknown";
  int cus = 0;
  if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) {
    std::snprintf(arch, sizeof(arch), "%s", prop.gcnArchName);
    cus = prop.multiProcessorCount;
  }
  for (char* c = arch; *c; ++c)
    if (*c == '"' || *c == '\\' || *c == '|' || (unsigned char)*c < 32) *c = '_';
  char key[256];
  std::snprintf(key, sizeof(key), "%s|%d|%dx%dx%d|k%d|v1", arch, cus, p->g.nx, p->g.ny, p->g.nz, inner);
  return key;
}

static bool json_int(const std::string& line, const char* name, int* out) {
  const std::string pat = std::string("\"") + name + "\":";
  const size_t at_ = line.find(pat);
  if (at_ == std::string::npos) return false;
  const char* b = line.c_str() + at_ + pat.size();
  char* e = nullptr;
  const long v = std::strtol(b, &e, 10);
  if (e == b || v < -2147483647L || v > 2147483647L) return false;
  *out = (int)v;
  return true;
}

static std::vector<std::string> read_lines(const char* path) {
  std::vector<std::string> lines;
  FILE* f = std::fopen(path, "r");
  if (!f) return lines;
  std::string cur;
  int ch;
  while ((ch = std::fgetc(f)) != EOF) {
    if (ch == '\n') {
      if (!cur.empty()) lines.push_back(cur);
      cur.clear();
    } else {
      cur.push_back((char)ch);
    }
  }
  if (!cur.empty()) lines.push_back(cur);
  std::fclose(f);
  return lines;
}

static std::string key_field(const std::string& key) { return "{\"key\": \"" + key + "\","; }

static bool cache_lookup(const char* path, const std::string& key, ri_tuning* out) {
  const std::string head = key_field(key);
  for (const std::string& line : read_lines(path)) {
    if (line.compare(0, head.size(), head) != 0) continue;
    ri_tuning t{};
    if (!json_int(line, "tv_levels", &t.tv_levels) || !json_int(line, "tv_blocks", &t.tv_blocks) ||
        !json_int(line, "col_blocks", &t.col_blocks))
      continue;
    if (t.tv_levels < kTvLevelsMin || t.tv_levels > kTvLevelsMax || t.tv_blocks < 64 || t.tv_blocks > 65536 ||
        t.col_blocks < kColMinBlocks || t.col_blocks > kColMaxBlocks)
      continue;
    *out = t;
    return true;
  }
  return false;
}

static bool cache_store(const char* path, const std::string& key, const ri_tuning& t, double best_ms,
                        double default_ms) {
  const std::string head = key_field(key);
  std::vector<std::string> lines;
  for (const std::string& line : read_lines(path))
    if (line.compare(0, head.size(), head) != 0) lines.push_back(line);
  char buf[512];
  std::snprintf(buf, sizeof(buf), "%s \"tv_levels\": %d, \"tv_blocks\": %d, \"col_blocks\": %d, "
                "\"best_ms\": %.6g, \"default_ms\": %.6g}", head.c_str(), t.tv_levels, t.tv_blocks, t.col_blocks,
                best_ms, default_ms);
  lines.push_back(buf);
  const std::string tmp = std::string(path) + ".tmp." + std::to_string((long)getpid());
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return false;
  bool ok = true;
  for (const std::string& line : lines) ok = ok && std::fprintf(f, "%s\n", line.c_str()) > 0;
  ok = (std::fclose(f) == 0) && ok;
  if (ok) ok = std::rename(tmp.c_str(), path) == 0;
  if (!ok) std::remove(tmp.c_str());
  return ok;
}

// Average device time of one call of `enq` on stream s: one untimed call, one
// timed call to size the repetition count (~5 ms of work, 3..50 calls).
template <class F>
static hipError_t time_calls(hipStream_t s, F&& enq, double* ms) {
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  float t = 0.f;
  int reps = 1;
  if (e == hipSuccess) e = enq();
  if (e == hipSuccess) e = hipEventRecord(a, s);
  if (e == hipSuccess) e = enq();
  if (e == hipSuccess) e = hipEventRecord(b, s);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
  if (e == hipSuccess) {
    reps = (int)std::min(50.0, std::max(3.0, std::ceil(5.0 / std::max(1e-3, (double)t))));
    e = hipEventRecord(a, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = enq();
    if (e == hipSuccess) e = hipEventRecord(b, s);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
  }
  if (a) hipEventDestroy(a);
  if (b) hipEventDestroy(b);
  *ms = (double)t / reps;
  return e;
}

extern "C" ri_status ri_plan_autotune(ri_plan* p, int32_t inner_iters, const char* cache_path, void* ws,
                                      size_t ws_bytes, void* stream, ri_autotune_report* report) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!p) return fail(RI_ERR_INVALID_ARG, "plan is NULL");
  if (inner_iters < 0) return fail(RI_ERR_INVALID_ARG, "inner_iters=%d must be >= 0", inner_iters);
  if (p->cplx) return fail(RI_ERR_INVALID_ARG, "RI_COMPLEX plans have no launch shapes to tune");
  if (p->dtype == RI_F64) return fail(RI_ERR_INVALID_ARG, "RI_F64 plans have no launch shapes to tune");
  const Layout LT = make_layout(p, RI_OP_AUTOTUNE);
  if (!ws) return fail(RI_ERR_INVALID_ARG, "workspace is NULL (needs %zu bytes)", LT.total);
  if (ws_bytes < LT.total) return fail(RI_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes < %zu required", ws_bytes, LT.total);
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != p->device) return fail(RI_ERR_INVALID_ARG, "plan belongs to device %d, current device is %d", p->device, dev);
  hipStream_t s = (hipStream_t)stream;
  ri_autotune_report rep{};
  const std::string key = tune_key(p, inner_iters);
  const ri_tuning dflt{kTvDefaultLevels, kTvDefaultBlocks, kColDefaultBlocks};
  auto finish = [&](const ri_tuning& t) {
    p->tune = t;
    drop_graph(p);
    rep.best = t;
    rep.tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (report) *report = rep;
    return RI_OK;
  };
  if (cache_path) {
    ri_tuning hit{};
    if (cache_lookup(cache_path, key, &hit)) {
      rep.from_cache = 1;
      return finish(hit);
    }
  }
  const int nx = p->g.nx, ny = p->g.ny, nz = p->g.nz;
  const size_t nvox = (size_t)nx * ny * nz;
  float* xv = at<float>(ws, LT.vol1);   // x for A, v for the prox (zeros)
  float* xo = at<float>(ws, LT.vol2);   // A^T y, prox output
  float* hy = at<float>(ws, LT.ax0);    // A x, y for A^T (zeros)
  HIP_TRY(launch_fill_f32(xv, nvox, 0.f, s));
  HIP_TRY(launch_fill_f32(hy, (size_t)nx * ny, 0.f, s));

  // column chunking: forward + adjoint
  std::vector<int> seen;
  std::vector<std::pair<int, double>> col_ms;
  double col_best = 0.0, col_dflt = 0.0;
  int col_choice = dflt.col_blocks;
  for (int c : kColBlockCands) {
    int nchunk = 0, ppc = 0;
    chunking(p, c, &nchunk, &ppc);
    if (std::find(seen.begin(), seen.end(), nchunk) != seen.end() && c != dflt.col_blocks) continue;
    seen.push_back(nchunk);
    const Layout L = make_layout(p, RI_OP_SOLVE, c);
    if (L.total > LT.total) continue;
    double ms = 0.0;
    HIP_TRY(time_calls(s, [&]() -> hipError_t {
      hipError_t e = enqueue_forward(p, L, ws, xv, hy, s);
      return e == hipSuccess ? enqueue_adjoint(p, L, ws, hy, xo, s) : e;
    }, &ms));
    ++rep.candidates;
    col_ms.push_back({c, ms});
    if (c == dflt.col_blocks) col_dflt = ms;
  }
  // keep the default unless a candidate beats it by 1 %, and a later candidate
  // only if it beats the kept one by 1 % (timing noise does not flip choices)
  col_best = col_dflt;
  for (const auto& cm : col_ms)
    if (cm.second < 0.99 * col_best) { col_best = cm.second; col_choice = cm.first; }

  // TV prox: fusion depth x z-chunking
  double tv_best = 0.0, tv_dflt = 0.0;
  std::vector<std::pair<std::pair<int, int>, double>> tv_ms;
  int lv_choice = dflt.tv_levels, tb_choice = dflt.tv_blocks;
  std::vector<std::pair<int, int>> seen_tv;
  for (int H = kTvLevelsMin; H <= kTvLevelsMax; ++H) {
    for (int b : kTvBlockCands) {
      const bool is_dflt = H == dflt.tv_levels && b == dflt.tv_blocks;
      const std::pair<int, int> g{H, tv_pass_zchunk(nx, ny, nz, H, b)};
      if (std::find(seen_tv.begin(), seen_tv.end(), g) != seen_tv.end() && !is_dflt) continue;
      seen_tv.push_back(g);
      ProxArgs a{};
      a.v = xv;
      a.x = xo;
      prox_duals(p, LT, ws, &a);
      a.rowflag = at<uint8_t>(ws, LT.rowflag);
      a.planeflag = at<uint8_t>(ws, LT.planeflag);
      a.nx = nx; a.ny = ny; a.nz = nz;
      a.inner_iters = inner_iters;
      a.nonneg = 1;
      a.step = 1.0 / p->lipschitz;
      a.l1 = 0.0;
      a.tv = 1.0;
      a.levels = H;
      a.blocks = b;
      double ms = 0.0;
      HIP_TRY(time_calls(s, [&]() -> hipError_t { return launch_prox(a, s, nullptr); }, &ms));
      ++rep.candidates;
      tv_ms.push_back({{H, b}, ms});
      if (is_dflt) tv_dflt = ms;
    }
  }
  tv_best = tv_dflt;
  for (const auto& tm : tv_ms)
    if (tm.second < 0.99 * tv_best) { tv_best = tm.second; lv_choice = tm.first.first; tb_choice = tm.first.second; }

  const ri_tuning best{lv_choice, tb_choice, col_choice};
  rep.default_ms = col_dflt + tv_dflt;
  rep.best_ms = col_best + tv_best;
  if (cache_path) rep.cache_written = cache_store(cache_path, key, best, rep.best_ms, rep.default_ms) ? 1 : -1;
  return finish(best);
}
