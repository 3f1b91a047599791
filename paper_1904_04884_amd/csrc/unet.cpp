// Warm-start 3D U-Net driver: parameter layout, activation / gradient buffers,
// forward, backward and Adam, behind the ri_unet_* C ABI.  All arithmetic runs
// in the kernels of unet.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/rihvr.h"
#include "unet_internal.h"

using namespace rihvr;

// error helper shared with abi.cpp
extern "C" const char* ri_last_error(void);
namespace rihvr {
ri_status set_error(ri_status st, const char* msg);
}

namespace {

enum Kind { CONV = 0, UP = 1, HEAD = 2 };

struct Layer {
  Kind kind;
  int cin, cout;
  size_t w, b;              // offsets in the FP32 parameter array
  size_t pf = 0, pb = 0;    // offsets of the packed forward / input-gradient BF16 weights
  int f_npad = 0, f_c = 0;  // forward GEMM: padded columns, channels per tap
  int b_npad = 0, b_c = 0;  // input-gradient GEMM
};

int pad(int v, int m) { return (v + m - 1) / m * m; }

struct Net {
  int L, base;
  std::vector<int> ch;
  std::vector<Layer> layers;  // order: enc{l}a, enc{l}b for l = 0..L-1; up{l}, dec{l}a, dec{l}b for l = L-2..0; head
  size_t nparams = 0, npacked = 0;
  int enc_a(int l) const { return 2 * l; }
  int enc_b(int l) const { return 2 * l + 1; }
  int up(int l) const { return 2 * L + 3 * (L - 2 - l); }
  int dec_a(int l) const { return up(l) + 1; }
  int dec_b(int l) const { return up(l) + 2; }
  int head() const { return (int)layers.size() - 1; }
};

Net build_net(int L, int base) {
  Net n;
  n.L = L;
  n.base = base;
  for (int l = 0; l < L; ++l) n.ch.push_back(base << l);
  auto add = [&](Kind k, int cin, int cout) {
    Layer y;
    y.kind = k;
    y.cin = cin;
    y.cout = cout;
    const size_t wsz = k == CONV ? (size_t)27 * cin * cout : k == UP ? (size_t)8 * cin * cout : (size_t)cin;
    y.w = n.nparams;
    n.nparams += wsz;
    y.b = n.nparams;
    n.nparams += (size_t)cout;
    if (k == CONV) {
      y.f_npad = pad(cout, 16);
      y.f_c = pad(cin, 8);
      y.b_npad = pad(cin, 16);
      y.b_c = pad(cout, 8);
      y.pf = n.npacked;
      n.npacked += (size_t)27 * y.f_npad * y.f_c;
      y.pb = n.npacked;
      n.npacked += (size_t)27 * y.b_npad * y.b_c;
    } else if (k == UP) {
      y.f_npad = 8 * cout;
      y.f_c = cin;
      y.b_npad = pad(cin, 16);
      y.b_c = cout;
      y.pf = n.npacked;
      n.npacked += (size_t)y.f_npad * y.f_c;
      y.pb = n.npacked;
      n.npacked += (size_t)8 * y.b_npad * y.b_c;
    } else {
      y.f_npad = 16;
      y.f_c = cin;
      y.b_npad = pad(cin, 16);
      y.b_c = 8;
      y.pf = n.npacked;
      n.npacked += (size_t)y.f_npad * y.f_c;
      y.pb = n.npacked;
      n.npacked += (size_t)y.b_npad * y.b_c;
    }
    n.layers.push_back(y);
  };
  int cin = 1;
  for (int l = 0; l < L; ++l) {
    add(CONV, cin, n.ch[l]);
    add(CONV, n.ch[l], n.ch[l]);
    cin = n.ch[l];
  }
  for (int l = L - 2; l >= 0; --l) {
    add(UP, n.ch[l + 1], n.ch[l]);
    add(CONV, 2 * n.ch[l], n.ch[l]);
    add(CONV, n.ch[l], n.ch[l]);
  }
  add(HEAD, n.ch[0], 1);
  return n;
}

// Activation / gradient buffers for one volume size.
struct Buffers {
  size_t total = 0;
  size_t packed = 0, in0 = 0, y = 0, gy8 = 0, loss = 0, part = 0;
  std::vector<size_t> a, cat, p, idx, da, db, ga, gcat, gda, gdb, gp;
  size_t bbot = 0, gbbot = 0;
};

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

Buffers layout(const Net& n, int D, int H, int W, bool train) {
  Buffers B;
  const int L = n.L;
  size_t off = 256;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  auto nv = [&](int l) { return (size_t)(D >> l) * (H >> l) * (W >> l); };
  B.packed = take(n.npacked * 2);
  B.in0 = take(nv(0) * 8 * 2);
  B.a.resize(L);
  B.cat.resize(L);
  B.p.resize(L);
  B.idx.resize(L);
  B.da.resize(L);
  B.db.resize(L);
  B.ga.resize(L);
  B.gcat.resize(L);
  B.gda.resize(L);
  B.gdb.resize(L);
  B.gp.resize(L);
  for (int l = 0; l < L; ++l) {
    const size_t c = n.ch[l];
    B.a[l] = take(nv(l) * c * 2);
    if (l < L - 1) {
      B.cat[l] = take(nv(l) * 2 * c * 2);
      B.p[l] = take(nv(l + 1) * c * 2);
      B.idx[l] = take(nv(l + 1) * c);
      B.da[l] = take(nv(l) * c * 2);
      B.db[l] = take(nv(l) * c * 2);
    }
  }
  B.bbot = take(nv(L - 1) * n.ch[L - 1] * 2);
  B.y = take(nv(0) * 4);
  if (train) {
    B.gy8 = take(nv(0) * 8 * 2);
    B.loss = take(4);
    for (int l = 0; l < L; ++l) {
      const size_t c = n.ch[l];
      B.ga[l] = take(nv(l) * c * 2);
      if (l < L - 1) {
        B.gcat[l] = take(nv(l) * 2 * c * 2);
        B.gda[l] = take(nv(l) * c * 2);
        B.gdb[l] = take(nv(l) * c * 2);
        B.gp[l] = take(nv(l + 1) * c * 2);
      }
    }
    B.gbbot = take(nv(L - 1) * n.ch[L - 1] * 2);
    // partial sums of the gradient reductions: the largest of any layer's
    // weight (chunks x taps x C x N), bias (chunks x N) and loss (blocks) partials
    size_t most = 16384;
    auto chunks = [](long rows, long per) { return (size_t)((rows + per - 1) / per); };
    for (int l = 0; l < L; ++l) {
      const long rows = (long)nv(l);
      const size_t c = n.ch[l], cin = l == 0 ? 1 : n.ch[l - 1];
      const size_t nw = chunks(rows, wgrad_rows_per_block(rows)), nbias = chunks(rows, bias_rows_per_block(rows));
      most = std::max(most, nw * 27 * std::max(cin, c) * c);               // encoder a, b
      most = std::max(most, nbias * 2 * c);
      if (l < L - 1) {
        most = std::max(most, nw * 27 * 2 * c * c);                           // decoder a (2c in), b
        const long crows = (long)nv(l + 1);
        const size_t nu = chunks(crows, wgrad_rows_per_block(crows));
        most = std::max(most, nu * 8 * (size_t)n.ch[l + 1] * c);              // up-convolution
      }
    }
    most = std::max(most, chunks((long)nv(0), wgrad_rows_per_block((long)nv(0))) * (size_t)n.ch[0]);   // head
    B.part = take(most * 4);
  }
  B.total = off;
  return B;
}

template <class T>
T* at(void* ws, size_t off) {
  const uintptr_t base = ((uintptr_t)ws + 255) & ~(uintptr_t)255;
  return reinterpret_cast<T*>(base + off - 256);
}

ri_status check_cfg(const ri_unet_config* c) {
  if (!c) return set_error(RI_ERR_INVALID_ARG, "unet config is NULL");
  // channel counts are padded to 16 * 2^k columns of MFMA tiles, which every
  // kernel case covers only for base = 8 * 2^k
  const bool pow2 = c->base >= 8 && (c->base & (c->base - 1)) == 0;
  if (c->levels < 1 || c->levels > 6 || !pow2 || (c->base << (c->levels - 1)) > 128)
    return set_error(RI_ERR_INVALID_ARG,
                     "unet config: levels in [1, 6], base one of 8, 16, 32, ..., base*2^(levels-1) <= 128");
  return RI_OK;
}

ri_status check_dims(const ri_unet_config* c, int D, int H, int W) {
  const int m = 1 << (c->levels - 1);
  if (D < m || H < m || W < m || D % m || H % m || W % m)
    return set_error(RI_ERR_UNSUPPORTED_SIZE, "unet volume dims must be positive multiples of 2^(levels-1)");
  return RI_OK;
}

#define UTRY(expr)                                                      \
  do {                                                                  \
    hipError_t e_ = (expr);                                             \
    if (e_ != hipSuccess) {                                             \
      char m_[256];                                                     \
      snprintf(m_, sizeof(m_), "%s: %s", #expr, hipGetErrorString(e_)); \
      return set_error(RI_ERR_HIP, m_);                                 \
    }                                                                   \
  } while (0)

GatherGemmArgs gemm(int mode, int D, int H, int W, const uint16_t* src, int cs, int c0, int T, int C,
                    const uint16_t* wt, int N, int Npad, const float* bias, int relu, void* dst, int dcs, int dc0,
                    int out_f32 = 0) {
  GatherGemmArgs g{};
  g.mode = mode;
  g.D = D; g.H = H; g.W = W;
  g.src = src; g.src_cs = cs; g.src_c0 = c0;
  g.T = T; g.C = C;
  g.wt = wt; g.N = N; g.Npad = Npad;
  g.bias = bias;
  g.relu = relu;
  g.out_f32 = out_f32;
  g.dst = dst; g.dst_cs = dcs; g.dst_c0 = dc0;
  return g;
}

ri_status pack_all(const Net& n, const float* params, uint16_t* packed, bool with_bwd, hipStream_t s) {
  for (const Layer& y : n.layers) {
    if (y.kind == CONV) {
      UTRY(launch_pack(params + y.w, 27, y.cin, y.cout, 1, y.f_npad, y.f_c, packed + y.pf, s));
      if (with_bwd) UTRY(launch_pack(params + y.w, 27, y.cin, y.cout, 0, y.b_npad, y.b_c, packed + y.pb, s));
    } else if (y.kind == UP) {
      UTRY(launch_pack_up_fwd(params + y.w, y.cin, y.cout, packed + y.pf, s));
      if (with_bwd) UTRY(launch_pack(params + y.w, 8, y.cin, y.cout, 0, y.b_npad, y.b_c, packed + y.pb, s));
    } else {
      UTRY(launch_pack(params + y.w, 1, y.cin, 1, 1, y.f_npad, y.f_c, packed + y.pf, s));
      if (with_bwd) UTRY(launch_pack(params + y.w, 1, y.cin, 1, 0, y.b_npad, y.b_c, packed + y.pb, s));
    }
  }
  return RI_OK;
}

ri_status forward(const Net& n, const float* params, const float* in, float scale, int D, int H, int W, void* ws,
                  const Buffers& B, bool train, hipStream_t s) {
  const int L = n.L;
  uint16_t* pk = at<uint16_t>(ws, B.packed);
  ri_status st = pack_all(n, params, pk, train, s);
  if (st != RI_OK) return st;
  uint16_t* in0 = at<uint16_t>(ws, B.in0);
  UTRY(launch_input(in, scale, in0, 8, (long)D * H * W, s));
  for (int l = 0; l < L; ++l) {
    const int Dl = D >> l, Hl = H >> l, Wl = W >> l, c = n.ch[l];
    const Layer& ea = n.layers[n.enc_a(l)];
    const Layer& eb = n.layers[n.enc_b(l)];
    const uint16_t* src = l == 0 ? in0 : at<uint16_t>(ws, B.p[l - 1]);
    const int scs = l == 0 ? 8 : n.ch[l - 1];
    uint16_t* a = at<uint16_t>(ws, B.a[l]);
    UTRY(launch_gather_gemm(gemm(GG_CONV3_FWD, Dl, Hl, Wl, src, scs, 0, 27, ea.f_c, pk + ea.pf, c, ea.f_npad,
                                 params + ea.b, 1, a, c, 0), s));
    uint16_t* bo = l < L - 1 ? at<uint16_t>(ws, B.cat[l]) : at<uint16_t>(ws, B.bbot);
    const int bcs = l < L - 1 ? 2 * c : c, bc0 = l < L - 1 ? c : 0;
    UTRY(launch_gather_gemm(gemm(GG_CONV3_FWD, Dl, Hl, Wl, a, c, 0, 27, eb.f_c, pk + eb.pf, c, eb.f_npad,
                                 params + eb.b, 1, bo, bcs, bc0), s));
    if (l < L - 1)
      UTRY(launch_pool_fwd(bo, bcs, bc0, at<uint16_t>(ws, B.p[l]), c, at<uint8_t>(ws, B.idx[l]), c, Dl / 2, Hl / 2,
                           Wl / 2, s));
  }
  const uint16_t* h = at<uint16_t>(ws, B.bbot);
  for (int l = L - 2; l >= 0; --l) {
    const int Dl = D >> l, Hl = H >> l, Wl = W >> l, c = n.ch[l], cu = n.ch[l + 1];
    const Layer& up = n.layers[n.up(l)];
    const Layer& da = n.layers[n.dec_a(l)];
    const Layer& db = n.layers[n.dec_b(l)];
    uint16_t* cat = at<uint16_t>(ws, B.cat[l]);
    GatherGemmArgs g = gemm(GG_UP_FWD, Dl / 2, Hl / 2, Wl / 2, h, cu, 0, 1, up.f_c, pk + up.pf, 8 * c, up.f_npad,
                            params + up.b, 0, cat, 2 * c, 0);
    g.up_cout = c;
    UTRY(launch_gather_gemm(g, s));
    uint16_t* dao = at<uint16_t>(ws, B.da[l]);
    UTRY(launch_gather_gemm(gemm(GG_CONV3_FWD, Dl, Hl, Wl, cat, 2 * c, 0, 27, da.f_c, pk + da.pf, c, da.f_npad,
                                 params + da.b, 1, dao, c, 0), s));
    uint16_t* dbo = at<uint16_t>(ws, B.db[l]);
    UTRY(launch_gather_gemm(gemm(GG_CONV3_FWD, Dl, Hl, Wl, dao, c, 0, 27, db.f_c, pk + db.pf, c, db.f_npad,
                                 params + db.b, 1, dbo, c, 0), s));
    h = dbo;
  }
  // head: ReLU output for inference; training keeps the pre-activation (the
  // loss is taken on it, so a voxel below zero still passes gradient)
  const Layer& hd = n.layers[n.head()];
  UTRY(launch_gather_gemm(gemm(GG_POINT, D, H, W, h, n.ch[0], 0, 1, hd.f_c, pk + hd.pf, 1, hd.f_npad, params + hd.b,
                               train ? 0 : 1, at<float>(ws, B.y), 1, 0, 1), s));
  return RI_OK;
}

WgradArgs wg(int mode, int D, int H, int W, const uint16_t* g, int gcs, int gc0, int N, const uint16_t* src,
             int scs, int sc0, int C, float* dw) {
  WgradArgs w{};
  w.mode = mode;
  w.D = D; w.H = H; w.W = W;
  w.g = g; w.g_cs = gcs; w.g_c0 = gc0; w.N = N; w.Npad = pad(N, 16);
  w.s = src; w.s_cs = scs; w.s_c0 = sc0; w.C = C; w.Cpad = pad(C, 16);
  w.dw = dw;
  w.rows_per_block = 2048;
  return w;
}

ri_status backward(const Net& n, const float* params, const float* target, float pos_weight, float* grads, int D,
                   int H, int W, void* ws, const Buffers& B, hipStream_t s) {
  const int L = n.L;
  uint16_t* pk = at<uint16_t>(ws, B.packed);
  const long nv0 = (long)D * H * W;
  uint16_t* gy8 = at<uint16_t>(ws, B.gy8);
  UTRY(launch_zero_u16(gy8, (size_t)nv0 * 8, s));
  float* part = at<float>(ws, B.part);
  UTRY(launch_mse(at<float>(ws, B.y), target, nv0, pos_weight, gy8, 8, at<float>(ws, B.loss), part, s));
  // head
  const Layer& hd = n.layers[n.head()];
  const uint16_t* top = L > 1 ? at<uint16_t>(ws, B.db[0]) : at<uint16_t>(ws, B.bbot);
  uint16_t* gtop = L > 1 ? at<uint16_t>(ws, B.gdb[0]) : at<uint16_t>(ws, B.gbbot);
  UTRY(launch_wgrad(wg(GG_POINT, D, H, W, gy8, 8, 0, 1, top, n.ch[0], 0, n.ch[0], grads + hd.w), 1, part, s));
  UTRY(launch_bias_grad(gy8, 8, 0, 1, nv0, grads + hd.b, part, s));
  UTRY(launch_gather_gemm(gemm(GG_POINT, D, H, W, gy8, 8, 0, 1, hd.b_c, pk + hd.pb, n.ch[0], hd.b_npad, nullptr, 0,
                               gtop, n.ch[0], 0), s));
  // decoder, finest level first
  for (int l = 0; l <= L - 2; ++l) {
    const int Dl = D >> l, Hl = H >> l, Wl = W >> l, c = n.ch[l], cu = n.ch[l + 1];
    const long nvl = (long)Dl * Hl * Wl;
    const Layer& up = n.layers[n.up(l)];
    const Layer& da = n.layers[n.dec_a(l)];
    const Layer& db = n.layers[n.dec_b(l)];
    uint16_t* gdb = at<uint16_t>(ws, B.gdb[l]);
    uint16_t* gda = at<uint16_t>(ws, B.gda[l]);
    uint16_t* gcat = at<uint16_t>(ws, B.gcat[l]);
    const uint16_t* dbo = at<uint16_t>(ws, B.db[l]);
    const uint16_t* dao = at<uint16_t>(ws, B.da[l]);
    const uint16_t* cat = at<uint16_t>(ws, B.cat[l]);
    UTRY(launch_relu_mask(gdb, c, 0, dbo, c, 0, c, nvl, s));
    UTRY(launch_wgrad(wg(GG_CONV3_FWD, Dl, Hl, Wl, gdb, c, 0, c, dao, c, 0, c, grads + db.w), 27, part, s));
    UTRY(launch_bias_grad(gdb, c, 0, c, nvl, grads + db.b, part, s));
    UTRY(launch_gather_gemm(gemm(GG_CONV3_BWD, Dl, Hl, Wl, gdb, c, 0, 27, db.b_c, pk + db.pb, c, db.b_npad, nullptr,
                                 0, gda, c, 0), s));
    UTRY(launch_relu_mask(gda, c, 0, dao, c, 0, c, nvl, s));
    UTRY(launch_wgrad(wg(GG_CONV3_FWD, Dl, Hl, Wl, gda, c, 0, c, cat, 2 * c, 0, 2 * c, grads + da.w), 27, part, s));
    UTRY(launch_bias_grad(gda, c, 0, c, nvl, grads + da.b, part, s));
    UTRY(launch_gather_gemm(gemm(GG_CONV3_BWD, Dl, Hl, Wl, gda, c, 0, 27, da.b_c, pk + da.pb, 2 * c, da.b_npad,
                                 nullptr, 0, gcat, 2 * c, 0), s));
    // up-convolution: gradient rows at the fine level, parameters over coarse rows
    const uint16_t* hin = (l + 1 == L - 1) ? at<uint16_t>(ws, B.bbot) : at<uint16_t>(ws, B.db[l + 1]);
    uint16_t* ghin = (l + 1 == L - 1) ? at<uint16_t>(ws, B.gbbot) : at<uint16_t>(ws, B.gdb[l + 1]);
    UTRY(launch_wgrad(wg(GG_UP_FWD, Dl / 2, Hl / 2, Wl / 2, gcat, 2 * c, 0, c, hin, cu, 0, cu, grads + up.w), 8, part, s));
    UTRY(launch_bias_grad(gcat, 2 * c, 0, c, nvl, grads + up.b, part, s));
    UTRY(launch_gather_gemm(gemm(GG_UP_BWD, Dl / 2, Hl / 2, Wl / 2, gcat, 2 * c, 0, 8, up.b_c, pk + up.pb, cu,
                                 up.b_npad, nullptr, 0, ghin, cu, 0), s));
  }
  // encoder, coarsest level first
  for (int l = L - 1; l >= 0; --l) {
    const int Dl = D >> l, Hl = H >> l, Wl = W >> l, c = n.ch[l];
    const long nvl = (long)Dl * Hl * Wl;
    const Layer& ea = n.layers[n.enc_a(l)];
    const Layer& eb = n.layers[n.enc_b(l)];
    uint16_t* gout = l == L - 1 ? at<uint16_t>(ws, B.gbbot) : at<uint16_t>(ws, B.gcat[l]);
    const uint16_t* out = l == L - 1 ? at<uint16_t>(ws, B.bbot) : at<uint16_t>(ws, B.cat[l]);
    const int ocs = l == L - 1 ? c : 2 * c, oc0 = l == L - 1 ? 0 : c;
    if (l < L - 1)
      UTRY(launch_pool_bwd(at<uint16_t>(ws, B.gp[l]), c, at<uint8_t>(ws, B.idx[l]), gout, ocs, oc0, c, Dl / 2,
                           Hl / 2, Wl / 2, s));
    UTRY(launch_relu_mask(gout, ocs, oc0, out, ocs, oc0, c, nvl, s));
    const uint16_t* a = at<uint16_t>(ws, B.a[l]);
    uint16_t* ga = at<uint16_t>(ws, B.ga[l]);
    UTRY(launch_wgrad(wg(GG_CONV3_FWD, Dl, Hl, Wl, gout, ocs, oc0, c, a, c, 0, c, grads + eb.w), 27, part, s));
    UTRY(launch_bias_grad(gout, ocs, oc0, c, nvl, grads + eb.b, part, s));
    UTRY(launch_gather_gemm(gemm(GG_CONV3_BWD, Dl, Hl, Wl, gout, ocs, oc0, 27, eb.b_c, pk + eb.pb, c, eb.b_npad,
                                 nullptr, 0, ga, c, 0), s));
    UTRY(launch_relu_mask(ga, c, 0, a, c, 0, c, nvl, s));
    const uint16_t* src = l == 0 ? at<uint16_t>(ws, B.in0) : at<uint16_t>(ws, B.p[l - 1]);
    const int scs = l == 0 ? 8 : n.ch[l - 1], cin = l == 0 ? 1 : n.ch[l - 1];
    UTRY(launch_wgrad(wg(GG_CONV3_FWD, Dl, Hl, Wl, ga, c, 0, c, src, scs, 0, cin, grads + ea.w), 27, part, s));
    UTRY(launch_bias_grad(ga, c, 0, c, nvl, grads + ea.b, part, s));
    if (l > 0)
      UTRY(launch_gather_gemm(gemm(GG_CONV3_BWD, Dl, Hl, Wl, ga, c, 0, 27, ea.b_c, pk + ea.pb, cin, ea.b_npad,
                                   nullptr, 0, at<uint16_t>(ws, B.gp[l - 1]), cin, 0), s));
  }
  return RI_OK;
}

// splitmix64 + Box-Muller, for parameter initialisation on the host
struct Rng {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
  double normal() { return std::sqrt(-2.0 * std::log(uniform())) * std::cos(2.0 * M_PI * uniform()); }
};

}  // namespace

extern "C" ri_status ri_unet_param_count(const ri_unet_config* cfg, size_t* n) {
  ri_status st = check_cfg(cfg);
  if (st != RI_OK) return st;
  if (!n) return set_error(RI_ERR_INVALID_ARG, "NULL output");
  *n = build_net(cfg->levels, cfg->base).nparams;
  return RI_OK;
}

extern "C" ri_status ri_unet_init_params(const ri_unet_config* cfg, uint64_t seed, float* params, void* stream) {
  ri_status st = check_cfg(cfg);
  if (st != RI_OK) return st;
  if (!params) return set_error(RI_ERR_INVALID_ARG, "params is NULL");
  const Net n = build_net(cfg->levels, cfg->base);
  std::vector<float> h(n.nparams);
  Rng r{seed};
  for (const Layer& y : n.layers) {
    const size_t wsz = y.b - y.w;
    const double sd = y.kind == CONV ? std::sqrt(2.0 / (27.0 * y.cin)) : std::sqrt(1.0 / y.cin);
    const bool head = &y == &n.layers[n.head()];
    // the head starts at zero weights: the first output is the bias everywhere
    for (size_t i = 0; i < wsz; ++i) h[y.w + i] = head ? 0.f : (float)(sd * r.normal());
    for (int i = 0; i < y.cout; ++i) h[y.b + i] = 0.01f;
  }
  UTRY(hipMemcpyAsync(params, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice, (hipStream_t)stream));
  UTRY(hipStreamSynchronize((hipStream_t)stream));
  return RI_OK;
}

extern "C" ri_status ri_unet_workspace_size(const ri_unet_config* cfg, int32_t d, int32_t h, int32_t w,
                                           int32_t training, size_t* bytes) {
  ri_status st = check_cfg(cfg);
  if (st != RI_OK) return st;
  st = check_dims(cfg, d, h, w);
  if (st != RI_OK) return st;
  if (!bytes) return set_error(RI_ERR_INVALID_ARG, "NULL output");
  *bytes = layout(build_net(cfg->levels, cfg->base), d, h, w, training != 0).total;
  return RI_OK;
}

extern "C" ri_status ri_unet_forward(const ri_unet_config* cfg, const float* params, const float* in, float scale,
                                     float* out, int32_t d, int32_t h, int32_t w, void* ws, size_t ws_bytes,
                                     void* stream) {
  ri_status st = check_cfg(cfg);
  if (st != RI_OK) return st;
  st = check_dims(cfg, d, h, w);
  if (st != RI_OK) return st;
  if (!params || !in || !out || !ws) return set_error(RI_ERR_INVALID_ARG, "NULL pointer");
  const Net n = build_net(cfg->levels, cfg->base);
  const Buffers B = layout(n, d, h, w, false);
  if (ws_bytes < B.total) return set_error(RI_ERR_WORKSPACE_TOO_SMALL, "unet workspace too small");
  hipStream_t s = (hipStream_t)stream;
  st = forward(n, params, in, scale, d, h, w, ws, B, false, s);
  if (st != RI_OK) return st;
  UTRY(hipMemcpyAsync(out, at<float>(ws, B.y), (size_t)d * h * w * sizeof(float), hipMemcpyDeviceToDevice, s));
  return RI_OK;
}

extern "C" ri_status ri_unet_train_step(const ri_unet_config* cfg, float* params, float* grads, float* adam_m,
                                        float* adam_v, int32_t step, float lr, const float* in, float scale,
                                        const float* target, float pos_weight, int32_t d, int32_t h, int32_t w,
                                        float* loss_out, void* ws, size_t ws_bytes, void* stream) {
  ri_status st = check_cfg(cfg);
  if (st != RI_OK) return st;
  st = check_dims(cfg, d, h, w);
  if (st != RI_OK) return st;
  if (!params || !grads || !in || !target || !ws || (lr > 0 && (!adam_m || !adam_v)))
    return set_error(RI_ERR_INVALID_ARG, "NULL pointer");
  if (lr > 0 && step < 1) return set_error(RI_ERR_INVALID_ARG, "Adam step must be >= 1");
  if (!(pos_weight > 0.f) || !std::isfinite(pos_weight))
    return set_error(RI_ERR_INVALID_ARG, "pos_weight must be finite and > 0");
  const Net n = build_net(cfg->levels, cfg->base);
  const Buffers B = layout(n, d, h, w, true);
  if (ws_bytes < B.total) return set_error(RI_ERR_WORKSPACE_TOO_SMALL, "unet workspace too small");
  hipStream_t s = (hipStream_t)stream;
  UTRY(hipMemsetAsync(grads, 0, n.nparams * sizeof(float), s));
  st = forward(n, params, in, scale, d, h, w, ws, B, true, s);
  if (st != RI_OK) return st;
  st = backward(n, params, target, pos_weight, grads, d, h, w, ws, B, s);
  if (st != RI_OK) return st;
  if (loss_out) UTRY(hipMemcpyAsync(loss_out, at<float>(ws, B.loss), sizeof(float), hipMemcpyDeviceToDevice, s));
  if (lr > 0) UTRY(launch_adam(params, grads, adam_m, adam_v, n.nparams, lr, 0.9, 0.999, 1e-8, step, s));
  return RI_OK;
}
