// Particle tracking back end on gfx950: segmentation of a reconstructed volume
// into objects and their weighted centroids (section "Methodology", the
// segmentation paragraph: a threshold at a small fraction of the maximum and a
// minimum object volume), linking of the objects of successive frames by the
// method of Crocker & Grier and track bookkeeping (section "Synthetic
// Turbulent Flow": weighted centroids, maximum displacement per frame,
// minimum track duration).
//
// Segmentation.  Voxels above rel * max(x) are foreground.  Connected
// components (26-connectivity) by union-find on a label array of one 32-bit
// word per voxel: every foreground voxel starts as its own root; each unites
// with its 13 foreground neighbours of smaller linear index, always linking
// the larger root below the smaller with an atomic minimum, so the root of a
// component ends as its smallest linear index.  Roots are then numbered in
// index order (per-block counts, one scan, per-block ranking); a root's label
// word takes its number with the top bit set, so any voxel finds its object
// number in two reads.  Per-object voxel counts and FP64 sums of x and x times
// each coordinate are accumulated with atomics; objects with at least
// min_voxels voxels are written in number order with their weighted centroid.
//
// Linking.  For two frames of object positions, the candidate links are the
// pairs within the maximum displacement (physical units through a per-axis
// spacing).  Sources that share candidate targets form subnetworks (union-find
// over sources and targets); a thread per subnetwork enumerates the
// assignments -- sources in ascending order, each taking one of its
// candidates by increasing distance or none, none last -- and keeps the first
// one of least sum(d^2) + max_disp^2 * (unlinked sources).  Distances and
// sums are formed with rounded FP64 operations in a fixed order, so equal
// costs resolve the same way on every run.
#include <hip/hip_runtime.h>

#include <cstdio>

#include "../../include/rihvr.h"

namespace rihvr {
ri_status set_error(ri_status st, const char* msg);
}

namespace {

constexpr uint32_t kBg = 0xffffffffu;        // background label
constexpr uint32_t kRootMark = 0x80000000u;  // a numbered root's label word
constexpr int kDetThreads = 256;
constexpr int kDetChunk = 4096;              // voxels per block of the numbering pass
constexpr int kLinkMaxCand = 8;              // candidates kept per source
constexpr int kLinkMaxSubnet = 8;            // sources per subnetwork

__device__ __forceinline__ uint32_t find_root(const uint32_t* lab, uint32_t i) {
  uint32_t p = lab[i];
  while (p != i) {
    i = p;
    p = lab[i];
  }
  return i;
}

// Link the components of a and b: the larger root is set below the smaller by
// an atomic minimum; when another thread relinked it first, retry from there.
__device__ __forceinline__ void unite(uint32_t* lab, uint32_t a, uint32_t b) {
  while (true) {
    a = find_root(lab, a);
    b = find_root(lab, b);
    if (a == b) return;
    if (a > b) {
      const uint32_t t = a;
      a = b;
      b = t;
    }
    const uint32_t old = atomicMin(&lab[b], a);
    if (old == b) return;
    b = old;
  }
}

// Clearing by a kernel rather than a memset, so that a caller may capture the
// sequence into a HIP graph.
__global__ void k_fill_u32(uint32_t* p, size_t n, uint32_t v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_det_max(const float* __restrict__ x, size_t n, uint32_t* maxbits) {
  __shared__ float red[kDetThreads / 64];
  float m = 0.f;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    m = fmaxf(m, x[i]);
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kDetThreads / 64; ++w) m = fmaxf(m, red[w]);
    atomicMax(maxbits, __float_as_uint(m));   // m >= 0: its bits order like the values
  }
}

__global__ void k_det_init(const float* __restrict__ x, size_t n, const uint32_t* maxbits, double rel,
                           uint32_t* __restrict__ lab) {
  const double thr = rel * (double)__uint_as_float(*maxbits);
  const bool any = __uint_as_float(*maxbits) > 0.f;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    lab[i] = (any && (double)x[i] > thr) ? (uint32_t)i : kBg;
}

__global__ void k_det_union(uint32_t* lab, int nx, int ny, int nz) {
  const size_t n = (size_t)nx * ny * nz;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    if (lab[i] == kBg) continue;
    const int x = (int)(i % nx), y = (int)((i / nx) % ny), z = (int)(i / ((size_t)nx * ny));
    // the 13 neighbours of smaller linear index
    for (int dz = -1; dz <= 0; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          if (dz == 0 && (dy > 0 || (dy == 0 && dx >= 0))) continue;
          const int zz = z + dz, yy = y + dy, xx = x + dx;
          if (zz < 0 || yy < 0 || yy >= ny || xx < 0 || xx >= nx) continue;
          const size_t j = ((size_t)zz * ny + yy) * nx + xx;
          if (lab[j] != kBg) unite(lab, (uint32_t)i, (uint32_t)j);
        }
  }
}

__global__ void k_det_compress(uint32_t* lab, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    if (lab[i] != kBg) lab[i] = find_root(lab, (uint32_t)i);
}

// Roots in each chunk of kDetChunk voxels.
__global__ void k_det_count_roots(const uint32_t* __restrict__ lab, size_t n, uint32_t* block_counts) {
  __shared__ uint32_t red[kDetThreads / 64];
  const size_t base = (size_t)blockIdx.x * kDetChunk;
  uint32_t c = 0;
  for (int k = threadIdx.x; k < kDetChunk; k += kDetThreads) {
    const size_t i = base + k;
    if (i < n && lab[i] == (uint32_t)i) ++c;
  }
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kDetThreads / 64; ++w) c += red[w];
    block_counts[blockIdx.x] = c;
  }
}

// Exclusive scan of m counts in place (one block); total -> *total.
__global__ void k_scan_counts(uint32_t* counts, int m, uint32_t* total) {
  __shared__ uint32_t part[kDetThreads];
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < m; base += kDetThreads) {
    const int i = base + threadIdx.x;
    const uint32_t v = i < m ? counts[i] : 0;
    part[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kDetThreads; off <<= 1) {   // inclusive Hillis-Steele scan
      const uint32_t t = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
      __syncthreads();
      part[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < m) counts[i] = carry + part[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 0) carry += part[kDetThreads - 1];
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

// Number the roots in index order; a root's label word becomes its number
// with the top bit set, and its index is recorded (numbers below max_comp).
__global__ void k_det_number(uint32_t* lab, size_t n, const uint32_t* __restrict__ offsets, uint32_t max_comp,
                             uint32_t* __restrict__ first) {
  __shared__ uint32_t wsum[kDetThreads / 64];
  const size_t base = (size_t)blockIdx.x * kDetChunk;
  uint32_t run = offsets[blockIdx.x];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int k = 0; k < kDetChunk; k += kDetThreads) {
    const size_t i = base + k + threadIdx.x;
    const bool root = i < n && lab[i] == (uint32_t)i;
    const uint64_t mask = __ballot(root);
    const uint32_t below = (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wv] = (uint32_t)__popcll(mask);
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (int w = 0; w < kDetThreads / 64; ++w) {
      before += w < wv ? wsum[w] : 0;
      tot += wsum[w];
    }
    if (root) {
      const uint32_t id = run + before + below;
      lab[i] = kRootMark | id;
      if (id < max_comp) first[id] = (uint32_t)i;
    }
    run += tot;
    __syncthreads();
  }
}

__device__ __forceinline__ uint32_t object_of(const uint32_t* lab, size_t i, uint32_t l) {
  return (l & kRootMark) ? (l & ~kRootMark) : (lab[l] & ~kRootMark);
}

__global__ void k_det_stats(const float* __restrict__ x, const uint32_t* __restrict__ lab, int nx, int ny, int nz,
                            uint32_t max_comp, uint32_t* cnt, double* sums /* [4][max_comp]: w, wz, wy, wx */) {
  const size_t n = (size_t)nx * ny * nz;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const uint32_t l = lab[i];
    if (l == kBg) continue;
    const uint32_t id = object_of(lab, i, l);
    if (id >= max_comp) continue;
    const double w = (double)x[i];
    const double px = (double)(i % nx), py = (double)((i / nx) % ny), pz = (double)(i / ((size_t)nx * ny));
    atomicAdd(&cnt[id], 1u);
    unsafeAtomicAdd(&sums[id], w);
    unsafeAtomicAdd(&sums[max_comp + id], w * pz);
    unsafeAtomicAdd(&sums[2 * (size_t)max_comp + id], w * py);
    unsafeAtomicAdd(&sums[3 * (size_t)max_comp + id], w * px);
  }
}

// Kept objects in number order (one block): out[k] = (z, y, x, w, count, first).
__global__ void k_det_finalize(const uint32_t* __restrict__ cnt, const double* __restrict__ sums,
                               const uint32_t* __restrict__ first, const uint32_t* ncomp_p, uint32_t max_comp,
                               int min_voxels, ri_object* out, int max_out, int32_t* counts) {
  __shared__ uint32_t wsum[kDetThreads / 64];
  const uint32_t ncomp = *ncomp_p;
  const uint32_t m = ncomp < max_comp ? ncomp : max_comp;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t run = 0;
  for (uint32_t base = 0; base < m; base += kDetThreads) {
    const uint32_t id = base + threadIdx.x;
    const bool keep = id < m && cnt[id] >= (uint32_t)min_voxels;
    const uint64_t mask = __ballot(keep);
    const uint32_t below = (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wv] = (uint32_t)__popcll(mask);
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (int w = 0; w < kDetThreads / 64; ++w) {
      before += w < wv ? wsum[w] : 0;
      tot += wsum[w];
    }
    if (keep) {
      const uint32_t k = run + before + below;
      if (k < (uint32_t)max_out) {
        const double w = sums[id];
        ri_object o;
        o.z = sums[max_comp + id] / w;
        o.y = sums[2 * (size_t)max_comp + id] / w;
        o.x = sums[3 * (size_t)max_comp + id] / w;
        o.weight = w;
        o.voxels = (double)cnt[id];
        o.first = (double)first[id];
        out[k] = o;
      }
    }
    run += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    counts[0] = (int32_t)run;
    counts[1] = (int32_t)ncomp;
  }
}

// ---------------------------------------------------------------------------
// Linking
// ---------------------------------------------------------------------------
struct LinkWs {
  int32_t* cand;      // [max_n0][kLinkMaxCand] target indices
  double* cand_d2;    // [max_n0][kLinkMaxCand]
  int32_t* ncand;     // [max_n0]
  uint32_t* parent;   // [max_n0 + max_n1] union-find over sources and targets
};

__device__ __forceinline__ double dist2(const ri_object& a, const ri_object& b, double sz, double sy, double sx) {
  // rounded FP64 products and sums in a fixed order (no contraction)
  const double dz = __dmul_rn(__dsub_rn(b.z, a.z), sz);
  const double dy = __dmul_rn(__dsub_rn(b.y, a.y), sy);
  const double dx = __dmul_rn(__dsub_rn(b.x, a.x), sx);
  return __dadd_rn(__dadd_rn(__dmul_rn(dz, dz), __dmul_rn(dy, dy)), __dmul_rn(dx, dx));
}

__global__ void k_link_candidates(const ri_object* __restrict__ prev, const int32_t* n0p, int max_n0,
                                  const ri_object* __restrict__ cur, const int32_t* n1p, int max_n1, double sz,
                                  double sy, double sx, double r2, LinkWs w, int32_t* link, int32_t* status) {
  const int n0 = min(*n0p, max_n0), n1 = min(*n1p, max_n1);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < max_n0 + max_n1; i += gridDim.x * blockDim.x)
    w.parent[i] = (uint32_t)i;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n0) return;
  link[i] = -1;
  int cj[kLinkMaxCand];
  double cd[kLinkMaxCand];
  int nc = 0, over = 0;
  const ri_object a = prev[i];
  for (int j = 0; j < n1; ++j) {
    const double d2 = dist2(a, cur[j], sz, sy, sx);
    if (!(d2 <= r2)) continue;
    // insert by (d2, j); j grows, so equal distances keep index order
    int k = nc < kLinkMaxCand ? nc : kLinkMaxCand - 1;
    if (nc == kLinkMaxCand) {
      over = 1;
      if (!(d2 < cd[kLinkMaxCand - 1])) continue;
    } else {
      ++nc;
    }
    while (k > 0 && d2 < cd[k - 1]) {
      cj[k] = cj[k - 1];
      cd[k] = cd[k - 1];
      --k;
    }
    cj[k] = j;
    cd[k] = d2;
  }
  if (over) atomicOr(status, 2);
  for (int k = 0; k < nc; ++k) {
    w.cand[(size_t)i * kLinkMaxCand + k] = cj[k];
    w.cand_d2[(size_t)i * kLinkMaxCand + k] = cd[k];
  }
  w.ncand[i] = nc;
}

__global__ void k_link_union(const int32_t* n0p, int max_n0, LinkWs w) {
  const int n0 = min(*n0p, max_n0);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n0) return;
  for (int k = 0; k < w.ncand[i]; ++k) unite(w.parent, (uint32_t)i, (uint32_t)(max_n0 + w.cand[(size_t)i * kLinkMaxCand + k]));
}

// One thread per subnetwork (its root is its smallest source): exhaustive
// search in the fixed enumeration order.
__global__ void k_link_solve(const int32_t* n0p, int max_n0, double r2, LinkWs w, int32_t* link, int32_t* status) {
  const int n0 = min(*n0p, max_n0);
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n0 || w.ncand[r] == 0 || find_root(w.parent, (uint32_t)r) != (uint32_t)r) return;
  int mem[kLinkMaxSubnet];
  int nm = 0;
  for (int s = r; s < n0; ++s) {
    if (w.ncand[s] == 0 || find_root(w.parent, (uint32_t)s) != (uint32_t)r) continue;
    if (nm == kLinkMaxSubnet) {
      atomicOr(status, 1);
      return;
    }
    mem[nm++] = s;
  }
  // depth-first over (source k, choice c): c < ncand takes candidate c, c == ncand leaves it unlinked
  int choice[kLinkMaxSubnet], best[kLinkMaxSubnet];
  double cost[kLinkMaxSubnet + 1];
  double best_cost = __builtin_huge_val();
  cost[0] = 0.0;
  int k = 0;
  choice[0] = -1;
  while (k >= 0) {
    const int s = mem[k];
    const int nc = w.ncand[s];
    int c = choice[k] + 1;
    // next admissible choice: a candidate not taken by an earlier source, or "none"
    for (; c < nc; ++c) {
      const int j = w.cand[(size_t)s * kLinkMaxCand + c];
      bool used = false;
      for (int q = 0; q < k; ++q)
        if (choice[q] < w.ncand[mem[q]] && w.cand[(size_t)mem[q] * kLinkMaxCand + choice[q]] == j) used = true;
      if (!used) break;
    }
    if (c > nc) {   // every choice of this source tried: back up
      --k;
      continue;
    }
    choice[k] = c;
    const double add = c < nc ? w.cand_d2[(size_t)s * kLinkMaxCand + c] : r2;
    const double cst = __dadd_rn(cost[k], add);
    if (cst >= best_cost) continue;   // no strictly better assignment below this one
    if (k + 1 == nm) {
      best_cost = cst;
      for (int q = 0; q < nm; ++q) best[q] = choice[q];
      continue;
    }
    cost[k + 1] = cst;
    ++k;
    choice[k] = -1;
  }
  for (int q = 0; q < nm; ++q) {
    const int s = mem[q];
    link[s] = best[q] < w.ncand[s] ? w.cand[(size_t)s * kLinkMaxCand + best[q]] : -1;
  }
}

// Track ids of the current frame from the links of the previous one (one
// block): linked particles keep their source's id, the others open new ids in
// ascending particle order; track lengths grow by one for every id present.
__global__ void k_track_update(const int32_t* __restrict__ link, const int32_t* n0p, const int32_t* __restrict__ ids_prev,
                               const int32_t* n1p, int max_n1, int32_t* ids, int32_t* next_id, int32_t* track_len,
                               int max_tracks) {
  __shared__ uint32_t wsum[kDetThreads / 64];
  const int n1 = min(*n1p, max_n1), n0 = *n0p;
  for (int j = threadIdx.x; j < n1; j += kDetThreads) ids[j] = -1;
  __syncthreads();
  for (int i = threadIdx.x; i < n0; i += kDetThreads) {
    const int j = link[i];
    if (j >= 0 && j < n1) ids[j] = ids_prev[i];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int start = *next_id;
  uint32_t run = 0;
  for (int base = 0; base < n1; base += kDetThreads) {
    const int j = base + threadIdx.x;
    const bool fresh = j < n1 && ids[j] < 0;
    const uint64_t mask = __ballot(fresh);
    const uint32_t below = (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wv] = (uint32_t)__popcll(mask);
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (int w = 0; w < kDetThreads / 64; ++w) {
      before += w < wv ? wsum[w] : 0;
      tot += wsum[w];
    }
    if (fresh) ids[j] = start + (int)(run + before + below);
    run += tot;
    __syncthreads();
  }
  for (int j = threadIdx.x; j < n1; j += kDetThreads) {
    const int id = ids[j];
    if (id < max_tracks) atomicAdd(&track_len[id], 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) *next_id = start + (int)run;
}

__global__ void k_track_filter(const int32_t* __restrict__ track_len, const int32_t* n_tracks_p, int max_tracks,
                               int min_len, uint8_t* kept, int32_t* n_kept) {
  const int n = min(*n_tracks_p, max_tracks);
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    const bool k = track_len[t] >= min_len;
    kept[t] = k ? 1 : 0;
    if (k) atomicAdd(n_kept, 1);
  }
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct DetLayout {
  size_t lab, maxbits, total, bcounts, first, cnt, sums, end;
  size_t nblk;
};

DetLayout det_layout(size_t n, size_t max_comp) {
  DetLayout L{};
  size_t off = 0;
  auto take = [&](size_t b) { const size_t o = off; off = align256(off + b); return o; };
  L.nblk = (n + kDetChunk - 1) / kDetChunk;
  L.lab = take(n * 4);
  L.maxbits = take(4);
  L.total = take(4);
  L.bcounts = take(L.nblk * 4);
  L.first = take(max_comp * 4);
  L.cnt = take(max_comp * 4);
  L.sums = take(max_comp * 4 * 8);
  L.end = off;
  return L;
}

size_t link_ws_bytes(int max_n0, int max_n1) {
  return align256((size_t)max_n0 * kLinkMaxCand * 4) + align256((size_t)max_n0 * kLinkMaxCand * 8) +
         align256((size_t)max_n0 * 4) + align256((size_t)(max_n0 + max_n1) * 4);
}

ri_status hip_fail(hipError_t e, const char* what) {
  char m[256];
  snprintf(m, sizeof(m), "%s: %s", what, hipGetErrorString(e));
  return rihvr::set_error(RI_ERR_HIP, m);
}

int grid_for(size_t n) {
  const size_t b = (n + kDetThreads - 1) / kDetThreads;
  return (int)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

}  // namespace

extern "C" ri_status ri_detect_workspace_size(int32_t nx, int32_t ny, int32_t nz, int32_t max_components,
                                              size_t* bytes) {
  if (!bytes) return rihvr::set_error(RI_ERR_INVALID_ARG, "bytes is NULL");
  if (nx < 1 || ny < 1 || nz < 1 || max_components < 1)
    return rihvr::set_error(RI_ERR_INVALID_ARG, "sizes and max_components must be >= 1");
  const size_t n = (size_t)nx * ny * nz;
  if (n > ((size_t)1 << 31)) return rihvr::set_error(RI_ERR_UNSUPPORTED_SIZE, "volumes above 2^31 voxels");
  *bytes = det_layout(n, (size_t)max_components).end + 256;
  return RI_OK;
}

extern "C" ri_status ri_detect(const ri_detect_params* prm, const float* x, int32_t nx, int32_t ny, int32_t nz,
                               ri_object* objects, int32_t max_objects, int32_t* counts, int32_t max_components,
                               void* ws, size_t ws_bytes, void* stream) {
  if (!prm || !x || !objects || !counts || !ws) return rihvr::set_error(RI_ERR_INVALID_ARG, "NULL argument");
  if (!(prm->rel_threshold >= 0.0) || prm->min_voxels < 1 || max_objects < 1)
    return rihvr::set_error(RI_ERR_INVALID_ARG, "rel_threshold >= 0, min_voxels >= 1, max_objects >= 1");
  size_t need = 0;
  ri_status st = ri_detect_workspace_size(nx, ny, nz, max_components, &need);
  if (st != RI_OK) return st;
  if (ws_bytes < need) return rihvr::set_error(RI_ERR_WORKSPACE_TOO_SMALL, "detect workspace too small");
  const size_t n = (size_t)nx * ny * nz;
  const DetLayout L = det_layout(n, (size_t)max_components);
  char* base = reinterpret_cast<char*>(((uintptr_t)ws + 255) & ~(uintptr_t)255);
  uint32_t* lab = reinterpret_cast<uint32_t*>(base + L.lab);
  uint32_t* maxbits = reinterpret_cast<uint32_t*>(base + L.maxbits);
  uint32_t* total = reinterpret_cast<uint32_t*>(base + L.total);
  uint32_t* bcounts = reinterpret_cast<uint32_t*>(base + L.bcounts);
  uint32_t* first = reinterpret_cast<uint32_t*>(base + L.first);
  uint32_t* cnt = reinterpret_cast<uint32_t*>(base + L.cnt);
  double* sums = reinterpret_cast<double*>(base + L.sums);
  hipStream_t s = (hipStream_t)stream;
  const uint32_t mc = (uint32_t)max_components;
  hipError_t e;
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, maxbits, (size_t)1, 0u);
  hipLaunchKernelGGL(k_det_max, dim3(grid_for(n)), dim3(kDetThreads), 0, s, x, n, maxbits);
  hipLaunchKernelGGL(k_det_init, dim3(grid_for(n)), dim3(kDetThreads), 0, s, x, n, maxbits, prm->rel_threshold, lab);
  hipLaunchKernelGGL(k_det_union, dim3(grid_for(n)), dim3(kDetThreads), 0, s, lab, nx, ny, nz);
  hipLaunchKernelGGL(k_det_compress, dim3(grid_for(n)), dim3(kDetThreads), 0, s, lab, n);
  hipLaunchKernelGGL(k_det_count_roots, dim3((unsigned)L.nblk), dim3(kDetThreads), 0, s, lab, n, bcounts);
  hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(kDetThreads), 0, s, bcounts, (int)L.nblk, total);
  hipLaunchKernelGGL(k_det_number, dim3((unsigned)L.nblk), dim3(kDetThreads), 0, s, lab, n, bcounts, mc, first);
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(mc)), dim3(kDetThreads), 0, s, cnt, (size_t)mc, 0u);
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for((size_t)mc * 8)), dim3(kDetThreads), 0, s,
                     reinterpret_cast<uint32_t*>(sums), (size_t)mc * 8, 0u);   // 4 x FP64 zeros per object
  hipLaunchKernelGGL(k_det_stats, dim3(grid_for(n)), dim3(kDetThreads), 0, s, x, lab, nx, ny, nz, mc, cnt, sums);
  hipLaunchKernelGGL(k_det_finalize, dim3(1), dim3(kDetThreads), 0, s, cnt, sums, first, total, mc, prm->min_voxels,
                     objects, max_objects, counts);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "detect launch");
  return RI_OK;
}

extern "C" ri_status ri_link_workspace_size(int32_t max_n0, int32_t max_n1, size_t* bytes) {
  if (!bytes || max_n0 < 1 || max_n1 < 1) return rihvr::set_error(RI_ERR_INVALID_ARG, "bad link sizes");
  *bytes = link_ws_bytes(max_n0, max_n1) + 256;
  return RI_OK;
}

extern "C" ri_status ri_link(const ri_object* prev, const int32_t* n_prev, int32_t max_prev, const ri_object* cur,
                             const int32_t* n_cur, int32_t max_cur, const double spacing[3], double max_disp,
                             int32_t* link, int32_t* status, void* ws, size_t ws_bytes, void* stream) {
  if (!prev || !n_prev || !cur || !n_cur || !spacing || !link || !status || !ws)
    return rihvr::set_error(RI_ERR_INVALID_ARG, "NULL argument");
  if (max_prev < 1 || max_cur < 1 || !(max_disp > 0.0) || !(spacing[0] > 0) || !(spacing[1] > 0) || !(spacing[2] > 0))
    return rihvr::set_error(RI_ERR_INVALID_ARG, "capacities >= 1, max_disp and spacing > 0");
  if (ws_bytes < link_ws_bytes(max_prev, max_cur) + 256)
    return rihvr::set_error(RI_ERR_WORKSPACE_TOO_SMALL, "link workspace too small");
  char* base = reinterpret_cast<char*>(((uintptr_t)ws + 255) & ~(uintptr_t)255);
  LinkWs w;
  size_t off = 0;
  w.cand = reinterpret_cast<int32_t*>(base + off);
  off += align256((size_t)max_prev * kLinkMaxCand * 4);
  w.cand_d2 = reinterpret_cast<double*>(base + off);
  off += align256((size_t)max_prev * kLinkMaxCand * 8);
  w.ncand = reinterpret_cast<int32_t*>(base + off);
  off += align256((size_t)max_prev * 4);
  w.parent = reinterpret_cast<uint32_t*>(base + off);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, reinterpret_cast<uint32_t*>(status), (size_t)1, 0u);
  const double r2 = max_disp * max_disp;
  const int nb = (max_prev + max_cur + kDetThreads - 1) / kDetThreads;
  hipLaunchKernelGGL(k_link_candidates, dim3(nb), dim3(kDetThreads), 0, s, prev, n_prev, max_prev, cur, n_cur, max_cur,
                     spacing[0], spacing[1], spacing[2], r2, w, link, status);
  const int nb0 = (max_prev + kDetThreads - 1) / kDetThreads;
  hipLaunchKernelGGL(k_link_union, dim3(nb0), dim3(kDetThreads), 0, s, n_prev, max_prev, w);
  hipLaunchKernelGGL(k_link_solve, dim3(nb0), dim3(kDetThreads), 0, s, n_prev, max_prev, r2, w, link, status);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "link launch");
  return RI_OK;
}

extern "C" ri_status ri_track_update(const int32_t* link, const int32_t* n_prev, const int32_t* ids_prev,
                                     const int32_t* n_cur, int32_t max_cur, int32_t* ids_cur, int32_t* next_id,
                                     int32_t* track_len, int32_t max_tracks, void* stream) {
  if (!n_prev || !n_cur || !ids_cur || !next_id || !track_len || max_cur < 1 || max_tracks < 1)
    return rihvr::set_error(RI_ERR_INVALID_ARG, "NULL argument or capacity < 1");
  hipLaunchKernelGGL(k_track_update, dim3(1), dim3(kDetThreads), 0, (hipStream_t)stream, link, n_prev, ids_prev, n_cur,
                     max_cur, ids_cur, next_id, track_len, max_tracks);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? RI_OK : hip_fail(e, "track launch");
}

extern "C" ri_status ri_track_filter(const int32_t* track_len, const int32_t* n_tracks, int32_t max_tracks,
                                     int32_t min_len, uint8_t* kept, int32_t* n_kept, void* stream) {
  if (!track_len || !n_tracks || !kept || !n_kept || max_tracks < 1)
    return rihvr::set_error(RI_ERR_INVALID_ARG, "NULL argument or capacity < 1");
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, s, reinterpret_cast<uint32_t*>(n_kept), (size_t)1, 0u);
  hipLaunchKernelGGL(k_track_filter, dim3((max_tracks + kDetThreads - 1) / kDetThreads), dim3(kDetThreads), 0, s,
                     track_len, n_tracks, max_tracks, min_len, kept, n_kept);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? RI_OK : hip_fail(e, "filter launch");
}
