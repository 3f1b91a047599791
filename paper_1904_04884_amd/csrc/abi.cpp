// C ABI of the library: argument validation, plans (FP64 tables), workspace
// layouts and the host side of the FISTA solve (kernel sequencing, HIP graph
// replay, stop-flag polling, phase timing).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
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
  int inner = -1, dense = -1, nonneg = -1;
};

struct ri_plan {
  ri_geometry g{};
  int m = 0;                 // nx / 2
  int device = 0;
  double lipschitz = 0.0;
  double* theta = nullptr;   // device [ny][m+1]
  double2* zc = nullptr;     // device [nz]
  float2* tw_row = nullptr;  // device [nx]
  float2* tw_col = nullptr;  // device [ny]
  int32_t* host_flag = nullptr;  // pinned, for stop polling
  hipStream_t capture = nullptr;
  GraphCache gc;
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
  if (p->host_flag) hipHostFree(p->host_flag);
  delete p;
}

static void twiddles(int n, std::vector<float2>& out) {
  out.resize(n);
  for (int k = 0; k < n; ++k) {
    // exp(-2 pi i k / n), angle reduced to the first half turn for accuracy
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
  if (g->flags & ~RI_NO_CARRIER) return fail(RI_ERR_INVALID_ARG, "unknown geometry flags 0x%x", g->flags);
  return RI_OK;
}

extern "C" ri_status ri_plan_create(const ri_geometry* g, ri_plan** out) {
  if (!out) return fail(RI_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  ri_status vs = validate_geometry(g);
  if (vs != RI_OK) return vs;
  ri_plan* p = new ri_plan();
  p->g = *g;
  p->m = g->nx / 2;
  const int nx = g->nx, ny = g->ny, nz = g->nz, m = p->m;
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) { free_plan(p); return fail(RI_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e)); }

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
    const double z = g->z0_um + g->dz_um * j;
    double c = 0.0;
    if (!(g->flags & RI_NO_CARRIER)) {
      const double t = z / g->wavelength_um;
      c = t - std::floor(t);
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
  size_t vol1 = 0, vol2 = 0, pa[3] = {0, 0, 0}, pb[3] = {0, 0, 0};  // volumes (float)
  size_t spec = 0, gp = 0, gi = 0, th = 0;                 // spectra (float2)
  size_t ax0 = 0, ax1 = 0;                                 // holograms (float)
  size_t rowflag = 0, planeflag = 0;                       // bytes
  size_t pdfit = 0, psum = 0, ptv = 0, hist = 0;           // doubles
  size_t state = 0;
  int nchunk = 1, ppc = 1;
  int n_dfit = 0, n_obj = 0;
};

static size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

static void chunking(const ri_plan* p, int* nchunk, int* ppc) {
  const int W = col_tile_width(p->g.ny);
  const int tiles = (p->m + W - 1) / W;
  int want = std::max(1, (512 + tiles - 1) / tiles);
  want = std::min(want, p->g.nz);
  const int per = (p->g.nz + want - 1) / want;
  *ppc = per;
  *nchunk = (p->g.nz + per - 1) / per;
}

static Layout make_layout(const ri_plan* p, ri_op op) {
  Layout L;
  const size_t nx = p->g.nx, ny = p->g.ny, nz = p->g.nz, m = p->m;
  const size_t vol = nx * ny * nz * sizeof(float);
  const size_t spec = m * ny * nz * sizeof(float2);
  const size_t hspec = m * ny * sizeof(float2);
  chunking(p, &L.nchunk, &L.ppc);
  size_t off = 256;  // slack so the base can be aligned up
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
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
    for (int k = 0; k < 3; ++k) L.pa[k] = take(vol);
    for (int k = 0; k < 3; ++k) L.pb[k] = take(vol);
  }
  if (op == RI_OP_SOLVE) {
    L.vol1 = take(vol);
    L.vol2 = take(vol);
    L.ax0 = take(nx * ny * sizeof(float));
    L.ax1 = take(nx * ny * sizeof(float));
    L.rowflag = take(ny * nz);
    L.planeflag = take(nz);
    L.n_dfit = (int)((ny + rows_per_block((int)m) - 1) / rows_per_block((int)m));
    L.n_obj = obj_blocks((int)nx, (int)ny, (int)nz);
    L.pdfit = take((size_t)L.n_dfit * sizeof(double));
    L.psum = take((size_t)L.n_obj * sizeof(double));
    L.ptv = take((size_t)L.n_obj * sizeof(double));
    L.hist = take((size_t)kHistCap * sizeof(double));
    L.state = take(sizeof(SolveState));
  }
  L.total = off;
  return L;
}

extern "C" ri_status ri_workspace_size(const ri_plan* p, ri_op op, size_t* bytes) {
  if (!p || !bytes) return fail(RI_ERR_INVALID_ARG, "NULL argument");
  if (op < RI_OP_FORWARD || op > RI_OP_SOLVE) return fail(RI_ERR_INVALID_ARG, "unknown op %d", (int)op);
  *bytes = make_layout(p, op).total;
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
  hipError_t e = launch_rows_r2c(m, ra, pt, s);
  if (e != hipSuccess) return e;
  FwdColsArgs fa{};
  fa.t = at<float2>(ws, L.spec);
  fa.gp = at<float2>(ws, L.gp);
  fa.m = m;
  fa.nz = nz;
  fa.planes_per_chunk = L.ppc;
  e = launch_fwd_cols(ny, L.nchunk, fa, pt, s);
  if (e != hipSuccess) return e;
  HoloColsInvArgs ha{at<float2>(ws, L.gp), at<float2>(ws, L.gi), m, L.nchunk, nullptr};
  e = launch_holo_cols_inv(ny, ha, pt, s);
  if (e != hipSuccess) return e;
  RowsC2RArgs ca{};
  ca.in = at<float2>(ws, L.gi);
  ca.nrows = ny;
  ca.out = out;
  ca.mode = 0;
  ca.scale = (float)(1.0 / ((double)p->g.nx * ny));
  return launch_rows_c2r(m, ca, pt, s);
}

extern "C" ri_status ri_forward(ri_plan* p, const float* x, float* b_out, void* ws, size_t ws_bytes,
                                void* stream) {
  if (!p) return fail(RI_ERR_INVALID_ARG, "plan is NULL");
  const size_t vb = (size_t)p->g.nx * p->g.ny * p->g.nz * sizeof(float), hb = (size_t)p->g.nx * p->g.ny * sizeof(float);
  ri_status st = check_common(p, x, b_out, ws, ws_bytes, RI_OP_FORWARD, vb, hb);
  if (st != RI_OK) return st;
  if (overlaps(x, vb, b_out, hb)) return fail(RI_ERR_INVALID_ARG, "x and b_out overlap");
  HIP_TRY(enqueue_forward(p, make_layout(p, RI_OP_FORWARD), ws, x, b_out, (hipStream_t)stream));
  return RI_OK;
}

extern "C" ri_status ri_adjoint(ri_plan* p, const float* y, float* x_out, void* ws, size_t ws_bytes, void* stream) {
  if (!p) return fail(RI_ERR_INVALID_ARG, "plan is NULL");
  const size_t vb = (size_t)p->g.nx * p->g.ny * p->g.nz * sizeof(float), hb = (size_t)p->g.nx * p->g.ny * sizeof(float);
  ri_status st = check_common(p, y, x_out, ws, ws_bytes, RI_OP_ADJOINT, hb, vb);
  if (st != RI_OK) return st;
  if (overlaps(y, hb, x_out, vb)) return fail(RI_ERR_INVALID_ARG, "y and x_out overlap");
  const Layout L = make_layout(p, RI_OP_ADJOINT);
  const PlanTables pt = p->tables();
  hipStream_t s = (hipStream_t)stream;
  const int ny = p->g.ny, nz = p->g.nz, m = p->m;
  RowsR2CArgs ra{};
  ra.x = y;
  ra.out = at<float2>(ws, L.th);
  ra.nrows = ny;
  ra.mode = 0;
  HIP_TRY(launch_rows_r2c(m, ra, pt, s));
  AdjColsArgs aa{at<float2>(ws, L.th), at<float2>(ws, L.spec), m, nz, L.ppc, nullptr};
  HIP_TRY(launch_adj_cols(ny, L.nchunk, aa, pt, s));
  AdjRowsArgs ar{};
  ar.u = at<float2>(ws, L.spec);
  ar.nrows = ny * nz;
  ar.ny = ny;
  ar.out = x_out;
  ar.mode = 0;
  ar.scale = (float)(1.0 / ((double)p->g.nx * ny));
  HIP_TRY(launch_adj_rows(m, ar, pt, s));
  return RI_OK;
}

extern "C" ri_status ri_prox_fused_lasso(ri_plan* p, const ri_prox_params* pp, double step, const float* v,
                                         float* x_out, void* ws, size_t ws_bytes, void* stream) {
  if (!p) return fail(RI_ERR_INVALID_ARG, "plan is NULL");
  if (!pp) return fail(RI_ERR_INVALID_ARG, "params is NULL");
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
  for (int k = 0; k < 3; ++k) a.pa[k] = at<float>(ws, L.pa[k]);
  for (int k = 0; k < 3; ++k) a.pb[k] = at<float>(ws, L.pb[k]);
  a.nx = p->g.nx;
  a.ny = p->g.ny;
  a.nz = p->g.nz;
  a.inner_iters = pp->inner_iters;
  a.nonneg = pp->nonneg ? 1 : 0;
  a.step = step;
  a.l1 = pp->l1;
  a.tv = pp->tv;
  HIP_TRY(launch_prox(a, (hipStream_t)stream, nullptr));
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
};

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

// One outer iteration: objective of x_it, momentum, gradient step, prox.
static hipError_t enqueue_iteration(const SolveCtx& c, hipStream_t s, PhaseTimer* tm) {
  ri_plan* p = c.p;
  const Layout& L = c.L;
  const PlanTables pt = p->tables();
  const int nx = p->g.nx, ny = p->g.ny, nz = p->g.nz, m = p->m;
  const float scale = (float)(1.0 / ((double)nx * ny));
  uint8_t* rowflag = at<uint8_t>(c.ws, L.rowflag);
  uint8_t* planeflag = at<uint8_t>(c.ws, L.planeflag);
  hipError_t e;
#define LTRY(x)                      \
  do {                               \
    e = (x);                         \
    if (e != hipSuccess) return e;   \
  } while (0)
  // objective pieces of x_it
  if (tm) tm->begin(PH_OBJ);
  ObjArgs oa{};
  oa.x0 = c.vol[0]; oa.x1 = c.vol[1]; oa.x2 = c.vol[2];
  oa.nx = nx; oa.ny = ny; oa.nz = nz;
  oa.rowflag = rowflag;
  oa.psum = at<double>(c.ws, L.psum);
  oa.ptv = at<double>(c.ws, L.ptv);
  oa.st = c.st;
  LTRY(launch_obj(oa, nullptr, s));
  if (tm) tm->end(1);
  // A x_it (skipping empty rows and planes unless dense)
  if (tm) tm->begin(PH_FORWARD);
  RowsR2CArgs ra{};
  for (int k = 0; k < 3; ++k) ra.xs[k] = c.vol[k];
  ra.out = at<float2>(c.ws, L.spec);
  ra.nrows = ny * nz;
  ra.rowflag = c.dense ? nullptr : rowflag;
  ra.st = c.st;
  ra.mode = 2;
  LTRY(launch_rows_r2c(m, ra, pt, s));
  FwdColsArgs fa{};
  fa.t = at<float2>(c.ws, L.spec);
  fa.gp = at<float2>(c.ws, L.gp);
  fa.m = m; fa.nz = nz; fa.planes_per_chunk = L.ppc;
  fa.rowflag = c.dense ? nullptr : rowflag;
  fa.planeflag = c.dense ? nullptr : planeflag;
  fa.st = c.st;
  LTRY(launch_fwd_cols(ny, L.nchunk, fa, pt, s));
  if (tm) tm->end(2);
  // hologram space: A x_it, data misfit, scalars, residual spectrum
  if (tm) tm->begin(PH_HOLO);
  HoloColsInvArgs ha{at<float2>(c.ws, L.gp), at<float2>(c.ws, L.gi), m, L.nchunk, c.st};
  LTRY(launch_holo_cols_inv(ny, ha, pt, s));
  RowsC2RArgs ca{};
  ca.in = at<float2>(c.ws, L.gi);
  ca.nrows = ny;
  ca.ax0 = at<float>(c.ws, L.ax0);
  ca.ax1 = at<float>(c.ws, L.ax1);
  ca.b = c.b;
  ca.partial = at<double>(c.ws, L.pdfit);
  ca.st = c.st;
  ca.mode = 1;
  ca.scale = scale;
  LTRY(launch_rows_c2r(m, ca, pt, s));
  ScalarArgs sa{};
  sa.st = c.st;
  sa.pdfit = at<double>(c.ws, L.pdfit);
  sa.n_dfit = L.n_dfit;
  sa.psum = at<double>(c.ws, L.psum);
  sa.ptv = at<double>(c.ws, L.ptv);
  sa.n_obj = L.n_obj;
  sa.hist = at<double>(c.ws, L.hist);
  LTRY(launch_scalars(sa, s));
  RowsR2CArgs rr{};
  rr.ax0 = at<float>(c.ws, L.ax0);
  rr.ax1 = at<float>(c.ws, L.ax1);
  rr.b = c.b;
  rr.out = at<float2>(c.ws, L.th);
  rr.nrows = ny;
  rr.st = c.st;
  rr.mode = 1;
  LTRY(launch_rows_r2c(m, rr, pt, s));
  if (tm) tm->end(4);
  // adjoint and gradient step: v = y - t A^T r over x_{it-1}
  if (tm) tm->begin(PH_ADJOINT);
  AdjColsArgs aa{at<float2>(c.ws, L.th), at<float2>(c.ws, L.spec), m, nz, L.ppc, c.st};
  LTRY(launch_adj_cols(ny, L.nchunk, aa, pt, s));
  AdjRowsArgs ar{};
  ar.u = at<float2>(c.ws, L.spec);
  ar.nrows = ny * nz;
  ar.ny = ny;
  ar.x0 = c.vol[0]; ar.x1 = c.vol[1]; ar.x2 = c.vol[2];
  ar.rowflag = rowflag;
  ar.planeflag = planeflag;
  ar.st = c.st;
  ar.step = c.step;
  ar.mode = 1;
  ar.scale = scale;
  LTRY(launch_adj_rows(m, ar, pt, s));
  if (tm) tm->end(2);
  // fused-lasso prox -> x_{it+1}, occupancy flags
  if (tm) tm->begin(PH_PROX);
  ProxArgs pa{};
  for (int k = 0; k < 3; ++k) pa.vol[k] = c.vol[k];
  for (int k = 0; k < 3; ++k) pa.pa[k] = at<float>(c.ws, L.pa[k]);
  for (int k = 0; k < 3; ++k) pa.pb[k] = at<float>(c.ws, L.pb[k]);
  pa.rowflag = rowflag;
  pa.planeflag = planeflag;
  pa.nx = nx; pa.ny = ny; pa.nz = nz;
  pa.inner_iters = c.inner;
  pa.nonneg = c.nonneg;
  pa.step = c.step;
  pa.l1 = c.l1;
  pa.tv = c.tv;
  pa.st = c.st;
  int nl = 0;
  LTRY(launch_prox(pa, s, &nl));
  if (tm) tm->end(nl);
#undef LTRY
  return hipSuccess;
}

static ri_status validate_solve(ri_plan* p, const ri_solve_params* sp, const float* b, float* x, void* ws,
                                size_t ws_bytes) {
  if (!p) return fail(RI_ERR_INVALID_ARG, "plan is NULL");
  if (!sp) return fail(RI_ERR_INVALID_ARG, "params is NULL");
  const size_t vb = (size_t)p->g.nx * p->g.ny * p->g.nz * sizeof(float), hb = (size_t)p->g.nx * p->g.ny * sizeof(float);
  ri_status st = check_common(p, b, x, ws, ws_bytes, RI_OP_SOLVE, hb, vb);
  if (st != RI_OK) return st;
  if (overlaps(b, hb, x, vb)) return fail(RI_ERR_INVALID_ARG, "b and x_inout overlap");
  if (!(sp->l1 >= 0) || !(sp->tv >= 0) || !std::isfinite(sp->l1) || !std::isfinite(sp->tv))
    return fail(RI_ERR_INVALID_ARG, "l1 and tv must be finite and >= 0");
  if (sp->max_iters < 0 || sp->inner_iters < 0) return fail(RI_ERR_INVALID_ARG, "iteration counts must be >= 0");
  if (sp->init != RI_INIT_ZERO && sp->init != RI_INIT_GIVEN) return fail(RI_ERR_INVALID_ARG, "init must be ZERO or GIVEN");
  if (sp->f_ref > 0 && !(sp->gap_tol >= 0)) return fail(RI_ERR_INVALID_ARG, "gap_tol must be >= 0");
  if (sp->flags & ~(RI_SOLVE_DENSE | RI_SOLVE_NO_GRAPH | RI_SOLVE_RESTART | RI_SOLVE_TIMING))
    return fail(RI_ERR_INVALID_ARG, "unknown solve flags 0x%x", sp->flags);
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
  if (sp->init == RI_INIT_ZERO) {
    if ((e = launch_fill_f32(c.vol[0], nvox, 0.f, s)) != hipSuccess) return e;
  } else {
    if ((e = launch_flags_from_x(c.vol[0], p->g.nx, p->g.ny, p->g.nz, rowflag, planeflag, s)) != hipSuccess) return e;
  }
  if ((e = launch_copy_f32(c.vol[2], c.vol[0], nvox, s)) != hipSuccess) return e;
  if ((e = launch_fill_f32(at<float>(c.ws, c.L.ax0), npix, 0.f, s)) != hipSuccess) return e;
  return launch_fill_f32(at<float>(c.ws, c.L.ax1), npix, 0.f, s);
}

static ri_status read_state(const SolveCtx& c, hipStream_t s, SolveState* out) {
  HIP_TRY(hipMemcpyAsync(out, c.st, sizeof(SolveState), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return RI_OK;
}

static ri_status get_graph(ri_plan* p, const SolveCtx& c, hipGraphExec_t* exec) {
  GraphCache& g = p->gc;
  if (g.exec && g.ws == c.ws && g.b == c.b && g.x == c.vol[0] && g.step == c.step && g.l1 == c.l1 &&
      g.tv == c.tv && g.inner == c.inner && g.dense == (int)c.dense && g.nonneg == c.nonneg) {
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
  g.inner = c.inner; g.dense = (int)c.dense; g.nonneg = c.nonneg;
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
  if (tm) tm->collect(rep->phase_ms, rep->phase_launches);
  return (ri_status)h.status;
}

extern "C" ri_status ri_solve(ri_plan* p, const ri_solve_params* sp, const float* b, float* x_inout, void* ws,
                              size_t ws_bytes, void* stream, ri_solve_report* report) {
  ri_status vs = validate_solve(p, sp, b, x_inout, ws, ws_bytes);
  if (vs != RI_OK) return vs;
  hipStream_t s = (hipStream_t)stream;
  SolveCtx c{};
  c.p = p;
  c.L = make_layout(p, RI_OP_SOLVE);
  c.ws = ws;
  c.b = b;
  c.vol[0] = x_inout;
  c.vol[1] = at<float>(ws, c.L.vol1);
  c.vol[2] = at<float>(ws, c.L.vol2);
  c.st = at<SolveState>(ws, c.L.state);
  c.step = 1.0 / p->lipschitz;
  c.l1 = sp->l1;
  c.tv = sp->tv;
  c.inner = sp->inner_iters;
  c.dense = (sp->flags & RI_SOLVE_DENSE) != 0;
  c.nonneg = sp->nonneg ? 1 : 0;
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
  const int every = std::max(1, sp->check_every);
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
  HIP_TRY(launch_copy_final(c.vol[0], c.vol[1], c.vol[2], x_inout, (size_t)p->g.nx * p->g.ny * p->g.nz, c.st, s));
  if (timing) tm.end(1);
  if (!report) return RI_OK;
  return fill_report(c, s, report, timing ? &tm : nullptr);
}

extern "C" ri_status ri_solve_batched(int32_t n, ri_plan* const* plans, const ri_solve_params* params,
                                      const float* const* b, float* const* x_inout, void* ws, size_t ws_bytes,
                                      void* stream, ri_solve_report* reports) {
  if (n < 0) return fail(RI_ERR_INVALID_ARG, "n < 0");
  if (n == 0) return RI_OK;
  if (!plans || !params || !b || !x_inout) return fail(RI_ERR_INVALID_ARG, "NULL array argument");
  size_t need = 0;
  std::vector<size_t> offs(n);
  for (int i = 0; i < n; ++i) {
    if (!plans[i]) return fail(RI_ERR_INVALID_ARG, "plans[%d] is NULL", i);
    offs[i] = need;
    need += align_up(make_layout(plans[i], RI_OP_SOLVE).total);
  }
  if (!ws) return fail(RI_ERR_INVALID_ARG, "workspace is NULL");
  if (ws_bytes < need) return fail(RI_ERR_WORKSPACE_TOO_SMALL, "workspace %zu bytes < %zu required", ws_bytes, need);
  for (int i = 0; i < n; ++i) {
    ri_status vs = validate_solve(plans[i], &params[i], b[i], x_inout[i], (char*)ws + offs[i],
                                  align_up(make_layout(plans[i], RI_OP_SOLVE).total));
    if (vs != RI_OK) return vs;
  }
  ri_status agg = RI_OK;
  for (int i = 0; i < n; ++i) {
    ri_status st = ri_solve(plans[i], &params[i], b[i], x_inout[i], (char*)ws + offs[i],
                            align_up(make_layout(plans[i], RI_OP_SOLVE).total), stream,
                            reports ? &reports[i] : nullptr);
    if (st != RI_OK && agg == RI_OK) agg = st;
  }
  return agg;
}
