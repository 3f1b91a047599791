// Internal declarations shared by the C ABI (host orchestration) and the HIP
// kernels.  Not part of the public interface.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/rihvr.h"

namespace rihvr {

// A pointer known to be the same in every lane (keeps address bases in SGPRs).
template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  const uint64_t u = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)u);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(u >> 32));
  return reinterpret_cast<T*>(((uint64_t)hi << 32) | lo);
}

// Workgroups are dispatched round-robin over the 8 XCDs in order of their
// linear id, and each XCD has its own L2.  xcd_tile maps the linear id to a
// work index such that every XCD gets one contiguous run of indices, so that
// neighbouring tiles (which share halo rows or cache lines) run on the same
// XCD at about the same time.  A bijection of [0, n).
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_tile(uint32_t id, uint32_t n) {
  const uint32_t q = n / kXcds, r = n % kXcds;   // XCD k runs q + (k < r) indices
  const uint32_t k = id % kXcds, j = id / kXcds;
  return k * q + min(k, r) + j;
}

// One of three buffers by a runtime slot index, chosen by selects among values
// already read (an indexed local array would be placed in scratch memory).
template <class T>
__device__ __forceinline__ T* pick3(T* a, T* b, T* c, int i) {
  a = uniform_ptr(a);
  b = uniform_ptr(b);
  c = uniform_ptr(c);
  return i == 0 ? a : (i == 1 ? b : c);
}

// Solver state that lives in device memory for the duration of a solve.  All
// control decisions (momentum, stop, buffer rotation) are taken on the device
// so that one iteration can be replayed as a HIP graph.
struct SolveState {
  int32_t it;          // index of the iterate evaluated by the next objective kernel
  int32_t done;        // 1: every kernel of the solve returns immediately
  int32_t converged;   // gap criterion met
  int32_t status;      // ri_status of the solve so far
  int32_t cur, prev, next;   // volume-buffer slots for the current iteration
  int32_t ax_cur, ax_prev;   // hologram-buffer slots
  int32_t max_iters;
  int32_t restart;
  int32_t scur;        // row store holding x_it (the other one: x_{it-1}, then x_{it+1})
  int32_t rows_peak;   // row stores: most pool rows any iterate took so far
  double s;            // FISTA s_k
  double beta;         // momentum of the current extrapolation
  double f_prev;       // objective of the previous iterate
  double f_first;      // F(x_0)
  double f_cur;        // objective of iterate `it`
  double gap;
  double f_ref, gap_tol;
  double l1, tv;
};

constexpr int kHistCap = 8192;   // objective history entries kept on the device

// Row-compressed storage of the solver's iterates in two alternating stores:
// x_k in store st->scur, x_{k-1} in the other one until the gradient step has
// read it, which is then cleared and receives x_{k+1}.  Only the rows holding
// a non-zero voxel are kept, in a pool of `cap` rows of nx floats;
// slot[k][row] is the pool row of a volume row (z * ny + y) or -1 for an
// all-zero row.  The final TV pass allocates a row when a segment first stores
// a non-zero value into it (claim of the slot, atomic counter, zero fill,
// publication); readers take a row from the pool or read zeros.  The gradient
// step's output v goes to a dense volume (the caller's x_inout).  on == 0:
// dense iterates (vol[3]).
struct RowStores {
  float* pool[2];
  int32_t* slot[2];     // [nz * ny]
  uint32_t* count;      // [2] pool rows taken
  uint32_t* overflow;   // set when a pool ran out of rows
  uint32_t cap;
  int nx;
  float* v;             // dense gradient-step output (the prox input)
  int on;
};

// Row `row` of store k, or nullptr when the row is all zero.
__device__ __forceinline__ const float* store_row(const RowStores& rs, int k, size_t row) {
  const int32_t* sl = k == 0 ? rs.slot[0] : rs.slot[1];
  float* pl = k == 0 ? rs.pool[0] : rs.pool[1];
  const int32_t s = sl[row];
  return s >= 0 ? pl + (size_t)s * rs.nx : nullptr;
}

// Device pointers of a plan's tables.
struct PlanTables {
  const double* theta;   // [ny][nx/2 + 1]  sqrt(1/lambda^2 - f^2) - 1/lambda  (FP64)
  const double2* zc;     // [nz] (z_j, carrier frac(z_j / lambda) or 0)
  const float2* tw_row;  // [nx]  exp(-2 pi i m / nx)
  const float2* tw_col;  // [ny]  exp(-2 pi i m / ny)
};

// Launch shapes (host side mirrors of the compile-time choices).
int rows_per_block(int m);     // rows of a length-m packed transform per row block
int col_tile_width(int ny);
// Default / largest target block count of the column transforms (z-chunking).
constexpr int kColDefaultBlocks = 512, kColMinBlocks = 16, kColMaxBlocks = 8192;    // columns per column tile
bool fft_len_supported(int L);

// ---------------------------------------------------------------------------
// Every kernel exists in two forms.  The single form runs one frame with the
// grid of that frame.  The batched form runs many frames (of one transform size
// where the kernel is specialised on a size) in one launch: the frames' block
// counts are laid end to end (prefix offsets offs[0..n], offs[0] = 0); block b
// finds its frame f with offs[f] <= b < offs[f+1], takes that frame's argument
// struct from a device array and decomposes b - offs[f] with the frame's grid
// (gx, gy), which the host writes into each struct.  Frames whose solve has
// stopped return at once.
// ---------------------------------------------------------------------------
struct BatchMap {
  const uint32_t* offs;  // device, n + 1 entries
  int n;
  // Persistent form (TV passes): kQueueWords words of claim counters, zero at
  // launch and zero again when the launch ends, and the blocks of the launch.
  uint32_t* queue = nullptr;
  int grid = 0;
};
// One counter per XCD range and one for the blocks that have finished, each
// on a 128-byte line of its own.
constexpr uint32_t kQueueStride = 32;
constexpr uint32_t kQueueWords = (kXcds + 1) * kQueueStride;

// Row-wise packed R2C of real rows [nrows][2m] -> [nrows][m] complex.  Rows with
// rowflag == 0 are skipped (nothing written).  mode 0: input x;  mode 1: input
// r = (1+beta) ax[cur] - beta ax[prev] - b computed on the fly (solver residual);
// mode 2: input xs[st->it % 3] (the solver iterate).
struct RowsR2CArgs {
  const float* x;            // mode 0 input
  const float* xs[3];        // mode 2 inputs
  const float* ax0; const float* ax1; const float* b;   // mode 1 inputs
  float2* out;
  int nrows;
  const uint8_t* rowflag;    // nullable
  const SolveState* st;      // nullable (mode 0 outside a solve)
  int mode;
  RowStores rs;              // mode 2 with rs.on: the iterate's rows come from its store
  PlanTables pt;
  int gx, gy;
};
dim3 grid_rows(int m, int nrows);
hipError_t launch_rows_r2c(int m, RowsR2CArgs a, hipStream_t s);
hipError_t launch_rows_r2c_batched(int m, const RowsR2CArgs* args, BatchMap map, int nblocks, hipStream_t s);

// Column FFT of the packed spectra of planes [z-chunk], multiply by cos(phase_j)
// and sum over the planes of the chunk -> partial spectra gp[chunk][ny][m].
struct FwdColsArgs {
  const float2* t;           // [nz][ny][m]
  float2* gp;                // [nchunk][ny][m]
  int m, nz, planes_per_chunk;
  const uint8_t* rowflag;    // nullable [nz][ny]
  const uint8_t* planeflag;  // nullable [nz]
  const SolveState* st;      // nullable
  PlanTables pt;
  int gx, gy;
};
dim3 grid_cols(int ny, int m, int nchunk);
hipError_t launch_fwd_cols(int ny, int nchunk, FwdColsArgs a, hipStream_t s);
hipError_t launch_fwd_cols_batched(int ny, const FwdColsArgs* args, BatchMap map, int nblocks, hipStream_t s);

// Sum of nchunk partial spectra, then unscaled inverse column FFT -> gi [ny][m].
struct HoloColsInvArgs {
  const float2* gp; float2* gi; int m, nchunk; const SolveState* st;
  PlanTables pt;
  int gx, gy;
};
hipError_t launch_holo_cols_inv(int ny, HoloColsInvArgs a, hipStream_t s);
hipError_t launch_holo_cols_inv_batched(int ny, const HoloColsInvArgs* args, BatchMap map, int nblocks,
                                        hipStream_t s);

// Row-wise packed C2R (scaled by 1/(nx ny)).  mode 0: write to out.  mode 1
// (solver): write ax[it & 1] and a per-block FP64 partial of 1/2 sum (ax - b)^2.
struct RowsC2RArgs {
  const float2* in; int nrows;
  float* out;                              // mode 0
  float* ax0; float* ax1; const float* b;  // mode 1
  double* partial;                         // mode 1: [nblocks]
  const SolveState* st;
  int mode;
  float scale;
  PlanTables pt;
  int gx, gy;
};
hipError_t launch_rows_c2r(int m, RowsC2RArgs a, hipStream_t s);
hipError_t launch_rows_c2r_batched(int m, const RowsC2RArgs* args, BatchMap map, int nblocks, hipStream_t s);

// Adjoint column pass: column FFT of the packed residual spectrum, then for each
// plane of the chunk multiply by cos(phase_j) and inverse column FFT -> u[j].
struct AdjColsArgs {
  const float2* th; float2* u; int m, nz, planes_per_chunk; const SolveState* st;
  PlanTables pt;
  int gx, gy;
};
hipError_t launch_adj_cols(int ny, int nchunk, AdjColsArgs a, hipStream_t s);
hipError_t launch_adj_cols_batched(int ny, const AdjColsArgs* args, BatchMap map, int nblocks, hipStream_t s);

// Adjoint row pass: packed C2R of u[j][y] scaled by 1/(nx ny).  mode 0: out = g.
// mode 1 (solver): v = y - step g with y = x[cur] + beta (x[cur] - x[prev]),
// written over x[prev]; also clears the row / plane occupancy flags.
struct AdjRowsArgs {
  const float2* u; int nrows, ny;
  float* out;                     // mode 0
  float* x0; float* x1; float* x2; // mode 1: the three rotating volume buffers
  uint8_t* rowflag; uint8_t* planeflag;
  uint8_t* rowflag_prev;          // mode 1, nullable: row flags of x_{k-1}; rows of x_k and
                                  // x_{k-1} with a clear flag are not read; set to x_k's
  const SolveState* st;
  double step;
  int mode;
  float scale;
  RowStores rs;                   // mode 1 with rs.on: x_k, x_{k-1} from their stores, v to rs.v
  PlanTables pt;
  int gx, gy;
};
hipError_t launch_adj_rows(int m, AdjRowsArgs a, hipStream_t s);
hipError_t launch_adj_rows_batched(int m, const AdjRowsArgs* args, BatchMap map, int nblocks, hipStream_t s);

// Objective pieces of a volume: per-block partials of sum(x) and TV3D(x).
struct ObjArgs {
  const float* x0; const float* x1; const float* x2; // slot st->it % 3 (or x0 when st null)
  int nx, ny, nz;
  const uint8_t* rowflag;     // nullable: skip rows whose neighbourhood is empty
  double* psum; double* ptv;  // [nblocks]
  const SolveState* st;
  int first_only;             // solver: only x_0 (later iterates are summed by the prox)
  int tv2;                    // per-plane 2D TV: no z differences
  RowStores rs;               // rs.on: x_it from store it & 1
  int gx, gy;
};
dim3 grid_obj(int nx, int ny, int nz);
int obj_blocks(int nx, int ny, int nz);
hipError_t launch_obj(ObjArgs a, hipStream_t s);
hipError_t launch_obj_batched(const ObjArgs* args, BatchMap map, int nblocks, hipStream_t s);

// FISTA scalars (one block per frame): reduce partials, objective, gap, stop
// flag, momentum, slots.
struct ScalarArgs {
  SolveState* st;
  const double* pdfit; int n_dfit;
  const double* psum; const double* ptv; int n_obj;      // objective partials of x_0
  const double* qsum; const double* qtv; int n_prox;     // ... of x_it, it > 0 (prox final pass)
  double* hist;   // [kHistCap]
  const uint32_t* overflow;   // nullable: a row store ran out of rows (the solve stops with an error)
  const uint32_t* count;      // nullable: rows taken in each row store (for the peak)
  int gx, gy;
};
hipError_t launch_scalars(ScalarArgs a, hipStream_t s);
hipError_t launch_scalars_batched(const ScalarArgs* args, BatchMap map, int nblocks, hipStream_t s);

// Number of frames of a batch whose solve has stopped -> *out (one block).
hipError_t launch_count_done(const SolveState* const* states, int n, int32_t* out, hipStream_t s);

struct StateInit {
  double f_ref, gap_tol, l1, tv;
  int32_t max_iters, restart;
};
hipError_t launch_state_init(SolveState* st, const StateInit& init, hipStream_t s);

// Utility kernels
hipError_t launch_fill_f32(float* p, size_t n, float v, hipStream_t s);
hipError_t launch_scale_f32(float* p, size_t n, float v, hipStream_t s);  // p *= v
hipError_t launch_fill_u8(uint8_t* p, size_t n, uint8_t v, hipStream_t s);
hipError_t launch_copy_f32(float* dst, const float* src, size_t n, hipStream_t s);
// Set row / plane flags of a volume from its contents (flags must be cleared).
hipError_t launch_flags_from_x(const float* x, int nx, int ny, int nz, uint8_t* rowflag,
                               uint8_t* planeflag, hipStream_t s);
// Copy the final iterate x[st->cur] into dst if it is not already there.
hipError_t launch_copy_final(const float* x0, const float* x1, const float* x2, float* dst,
                             size_t n, const SolveState* st, hipStream_t s);
// Row stores: dense copy of store st->scur (all-zero rows written as zeros);
// compress a dense volume into store 0 and duplicate it into store 1 (the start
// x_0 = x_{-1}); clear store st->scur ^ 1 before the prox writes x_{k+1} to it.
hipError_t launch_store_expand(const RowStores& rs, float* dst, int ny, int nz, const SolveState* st, hipStream_t s);
hipError_t launch_store_start(const RowStores& rs, const float* x, int ny, int nz, hipStream_t s);
hipError_t launch_store_clear_next(const RowStores& rs, int ny, int nz, const SolveState* st, hipStream_t s);

// Lipschitz constant on the device: max_f sum_j cos^2(phase_j(f)) in FP64.
hipError_t launch_lipschitz(const PlanTables& pt, int m, int ny, int nz, double* partial_max,
                            int* nblocks, hipStream_t s);

// ---------------------------------------------------------------------------
// Fused-lasso prox (tv.hip)
// ---------------------------------------------------------------------------
struct ProxArgs {
  const float* v;      // input volume (solver: slot st->prev)
  float* x;            // output volume (solver: slot st->next)
  float* vol[3];       // solver: the rotating volume buffers (v and x chosen on device)
  float* pa[3];        // dual components px, py, pz (ping)
  float* pb[3];        // dual components (pong)
  float* pa2[3];       // FGP: the second dual of each set (p beside r)
  float* pb2[3];
  uint8_t* rowflag; uint8_t* planeflag;  // nullable: set where x != 0
  double* psum; double* ptv;             // nullable: per-block sum(x), TV(x) of the result
  int nx, ny, nz;
  int inner_iters;
  int nonneg;
  double step, l1, tv;   // outside a solve (st == nullptr)
  const SolveState* st;  // solver: weights from st, step from `step`
  int levels;            // dual steps fused per pass (kTvLevelsMin..kTvLevelsMax; else the default)
  int blocks;            // target blocks per pass (<= 0: the default)
  int tv2;               // per-plane 2D TV (pa[2], pb[2] unused)
  int cus;               // compute units of the device (shapes the final pass's grid; <= 0: uniform)
  int dual_bf16;         // dual buffers hold bfloat16
  int fgp;               // accelerated dual iteration (one step per pass; pa2 / pb2 hold p)
  RowStores rs;          // solver with rs.on: v from rs.v, x_{k+1} into store st->scur ^ 1
  int warm;              // solver: the dual starts from the previous prox's (kept in pa / pb,
                         // the sets alternating by outer iteration when the pass count is odd)
  int group_planes;      // per-plane 2D TV: prox G planes at a time, pa / pb holding G planes (0: all)
  float* stage_group;    // grouped prox in place: each group's x is written here (G planes) and
                         // then copied over v (nullable)
};
constexpr int kTvLevelsMin = 2, kTvLevelsMax = 4, kTvDefaultLevels = 3;
constexpr int kTvDefaultBlocks = 1536;
hipError_t launch_prox(const ProxArgs& a, hipStream_t s, int* launches);
int prox_passes(int inner_iters, double tau, int levels, bool fgp);
int prox_levels(int levels, bool fgp);
// Planes per block of a pass for the given tuning (distinct values = distinct grids).
int tv_pass_zchunk(int nx, int ny, int nz, int levels, int blocks);
// Blocks of a dual pass and of the final pass (its tiles have a halo one
// wider) for the given tuning, and a bound over every tuning and pass.
int tv_pass_blocks(int nx, int ny, int nz, int levels, int blocks);
int tv_final_blocks(int nx, int ny, int nz, int levels, int blocks, int cus);
int tv_blocks_bound(int nx, int ny, int nz, int cus);
// Grouped per-plane prox: final-pass blocks of all groups of G planes (the
// objective partials of group g start at the sum over the groups before it),
// and a bound over every tuning.
int tv_group_final_blocks(int nx, int ny, int nz, int G, int levels, int blocks, int cus);
int tv_group_blocks_bound(int nx, int ny, int nz, int G, int cus);

// Batched prox: the argument structs of every pass of every frame are built on
// the host (prox_pass_args) and uploaded; launch p runs pass p of all frames.
struct TvPassArgs;
size_t tv_pass_args_size();
// Fills `out` (npass structs, host memory of npass * tv_pass_args_size() bytes)
// for one frame and returns the number of passes; blocks_per_pass (nullable,
// npass entries) receives the frame's blocks of each pass.
int prox_pass_args(const ProxArgs& a, void* out, int* blocks_per_pass);
hipError_t launch_tv_pass_batched(int levels, bool final_pass, bool tv2, bool fgp, bool bf16, bool sparse,
                                  const void* args, BatchMap map, int nblocks, hipStream_t s);

// Complex-valued object (cplx.hip): volumes [2][nz/2][ny][nx] (real parts, then
// imaginary parts; `nz` in the argument structs counts the planes of both).
// The fused-lasso prox with the complex TV (GP on a complex dual, pa[] and
// pb[] the two dual sets, alternating step by step) and the complex shrinkage; the solver's
// objective partials of sum |x| and the complex TV in `nblocks` blocks.
hipError_t launch_cprox(const ProxArgs& a, hipStream_t s, int* launches);
hipError_t launch_cobj(const ObjArgs& a, int nblocks, hipStream_t s);

// FP64 plans (f64.hip, cplx.hip): plain complex transforms of whole planes,
// the filter from the same FP64 tables; unfused gradient-projection prox.
struct Plan64Tables {
  const double* theta;   // [ny][nx/2 + 1]
  const double2* zc;     // [nzp] (z_j, carrier phase c_j)
  const double2* tw_x;   // [nx] exp(-2 pi i k / nx)
  const double2* tw_y;   // [ny]
  int nx, ny, m, nzp;    // nzp: planes of every part together
};
size_t f64_spectra_bytes(const Plan64Tables& t);
// b = A x (x: [nzp][ny][nx], b: [ny][nx]); X: [nzp][ny][nx] complex scratch,
// S: [ny][nx] complex scratch.
hipError_t forward64(const Plan64Tables& t, const double* x, double* b, double2* X, double2* S, hipStream_t s);
// x = A^T y, same scratch.
hipError_t adjoint64(const Plan64Tables& t, const double* y, double* x, double2* X, double2* S, hipStream_t s);
hipError_t axpby64(double* out, double a, const double* x, double b, const double* y, size_t n, hipStream_t s);
hipError_t fill64(double* out, double v, size_t n, hipStream_t s);
// per-block partials of sum (x - y)^2 in part[nblocks]
hipError_t sqdist64(const double* x, const double* y, size_t n, double* part, int nblocks, hipStream_t s);
struct Prox64Args {
  const double* v; double* x;   // [parts][nz][ny][nx]; x may be v
  double* p[3];                 // dual components, as v (p[2] unused in 2D)
  double* p2[3];                // the second dual set (the sets alternate step by step)
  int nx, ny, nz;               // nz: planes of one part
  int parts;                    // 1: real object, 2: complex object
  int tv2, nonneg, inner_iters;
  double step, l1, tv;
};
hipError_t launch_prox64(const Prox64Args& a, hipStream_t s);
// per-block partials of sum |x| and TV(x) in psum / ptv [nblocks]
hipError_t launch_obj64(const double* x, int nx, int ny, int nz, int parts, int tv2, double* psum, double* ptv,
                        int nblocks, hipStream_t s);

}  // namespace rihvr
