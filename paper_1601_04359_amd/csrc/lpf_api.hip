// liblpf C ABI: argument checks, per-context caches and scratch, launch plans.
// Declarations and the contract of every entry point are in include/lpf.h.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <queue>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/lpf.h"
#include "lpf_internal.h"

using namespace lpf;

namespace {

thread_local std::string g_err;

lpf_status fail(lpf_status s, const std::string &msg) {
  g_err = msg;
  return s;
}

lpf_status hip_fail(hipError_t e, const char *what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? LPF_E_NOMEM : LPF_E_DEVICE;
}

// Makes the context's device current for the scope and restores the caller's device.
struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

// Device buffer that only grows.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  hipError_t ensure(size_t n) {
    if (n <= bytes) return hipSuccess;
    if (p) {
      hipError_t e = hipFree(p);
      p = nullptr;
      bytes = 0;
      if (e != hipSuccess) return e;
    }
    hipError_t e = hipMalloc(&p, n);
    if (e == hipSuccess) bytes = n;
    return e;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
};

struct FullPlan {
  FullShape sh{};
  VecDesc *vecs = nullptr;   // device, bin order
  int32_t *bin_off = nullptr;  // device, nbins + 1
  int16_t *dxdy = nullptr;   // device, canonical order
  int64_t nv = 0;
};

// Canonical half domain (eq. (segments) with a cutoff, one of each {v, -v}).
void canonical_vectors(int cx, int cy, std::vector<int16_t> &out) {
  out.clear();
  out.reserve(2 * ((size_t)(cx + 1) * (cy + 1) + (size_t)cx * cy));
  for (int dy = 0; dy <= cy; ++dy)
    for (int dx = 0; dx <= cx; ++dx) {
      out.push_back((int16_t)dx);
      out.push_back((int16_t)dy);
    }
  for (int dy = 1; dy <= cy; ++dy)
    for (int dx = -cx; dx < 0; ++dx) {
      out.push_back((int16_t)dx);
      out.push_back((int16_t)dy);
    }
}

int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

// LDS bank-conflict score of a row stride: worst bank multiplicity of one wave's first dword
// read, for 32 and for 64 banks.
int bank_score(int rst, int R, int S) {
  const int rpw = 64 / S;
  int worst = 0;
  for (int banks : {32, 64}) {
    for (int half = 0; half < 64; half += banks) {
      std::vector<int> cnt(banks, 0);
      for (int l = half; l < half + banks && l < 64; ++l) {
        const int strip = l / rpw, r_in = l - strip * rpw;
        const int b = (r_in * rst + strip * R) % banks;
        worst = std::max(worst, ++cnt[b]);
      }
    }
  }
  return worst;
}

constexpr int kMaxLds = 160 * 1024;

}  // namespace

struct lpf_ctx_s {
  int dev = 0;
  std::map<std::tuple<int, int, int, int, int, int, int>, FullPlan> full_plans;
  DevBuf ext, part;
  std::mutex mu;
  // shape override (autotuner): R, S, wpg, lds budget; 0 = automatic
  int force_R = 0, force_S = 0, force_wpg = 0, force_lds = 0;
};

namespace {

bool choose_shape(lpf_ctx c, int W, int H, int cx, int cy, FullShape &sh, std::string &why) {
  const int swd = (W + 31) / 32;
  int R = c->force_R ? c->force_R : std::min(8, next_pow2(swd));
  int S = c->force_S ? c->force_S : next_pow2((swd + R - 1) / R);
  if (S > 64) {
    why = "image too wide for the lane layout (W > 64*R*32)";
    return false;
  }
  if ((long)R * S < swd) {
    why = "forced tile shape does not cover the row";
    return false;
  }
  const int rpw = 64 / S;
  sh.R = R;
  sh.S = S;
  sh.wpg = c->force_wpg ? c->force_wpg : 8;
  sh.we = S * R + (cx >> 5) + 1;
  int best = sh.we, best_score = 1 << 30;
  for (int r = sh.we; r < sh.we + 64; ++r) {
    int sc = bank_score(r, R, S);
    if (sc < best_score) {
      best_score = sc;
      best = r;
    }
  }
  sh.rst = best;
  int budget = c->force_lds ? c->force_lds : 64 * 1024;
  for (;;) {
    const int rows_max = budget / (sh.rst * 4);
    int tile = rows_max - cy - rpw;
    if (tile >= H) {
      tile = H;
    } else {
      tile = (tile / rpw) * rpw;
    }
    if (tile >= 1) {
      sh.tile = tile;
      break;
    }
    if (budget >= kMaxLds) {
      why = "cutoff cy too large for on-chip staging of the halo rows";
      return false;
    }
    budget = kMaxLds;
  }
  sh.ntiles = (H + sh.tile - 1) / sh.tile;
  sh.lds_rows = sh.tile + cy + rpw;
  return true;
}

lpf_status get_full_plan(lpf_ctx c, int W, int H, int cx, int cy, FullPlan *&plan) {
  FullShape sh{};
  std::string why;
  if (!choose_shape(c, W, H, cx, cy, sh, why)) return fail(LPF_E_UNSUPPORTED, "lpf_full: " + why);
  auto key = std::make_tuple(W, H, cx, cy, sh.R * 1000 + sh.S, sh.wpg, sh.tile);
  auto it = c->full_plans.find(key);
  if (it != c->full_plans.end()) {
    plan = &it->second;
    return LPF_OK;
  }
  std::vector<int16_t> can;
  canonical_vectors(cx, cy, can);
  const int64_t nv = (int64_t)can.size() / 2;
  if (nv > (int64_t)1 << 30) return fail(LPF_E_UNSUPPORTED, "lpf_full: too many vectors");

  // Wave-level bins, longest-processing-time-first on cost = pixels + per-band overhead.
  const int64_t target = std::max<int64_t>(sh.wpg, 8192 / sh.ntiles);
  int64_t nb = std::min<int64_t>(nv, target);
  nb = (nb + sh.wpg - 1) / sh.wpg * sh.wpg;
  sh.nbins = (int)nb;
  std::vector<int> order(nv);
  std::vector<int> cost(nv);
  for (int64_t i = 0; i < nv; ++i) {
    order[i] = (int)i;
    const int adx = std::abs((int)can[2 * i]), ady = std::abs((int)can[2 * i + 1]);
    cost[i] = std::max(adx, ady) + 1 + 2;
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  using Item = std::pair<int64_t, int>;  // (load, bin)
  std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
  for (int b = 0; b < sh.nbins; ++b) heap.push({0, b});
  std::vector<std::vector<int>> bins(sh.nbins);
  for (int i : order) {
    Item t = heap.top();
    heap.pop();
    bins[t.second].push_back(i);
    heap.push({t.first + cost[i], t.second});
  }
  std::vector<VecDesc> vecs;
  vecs.reserve(nv);
  std::vector<int32_t> off(sh.nbins + 1, 0);
  for (int b = 0; b < sh.nbins; ++b) {
    off[b] = (int32_t)vecs.size();
    for (int i : bins[b]) vecs.push_back(VecDesc{can[2 * i], can[2 * i + 1], i});
  }
  off[sh.nbins] = (int32_t)vecs.size();

  FullPlan p;
  p.sh = sh;
  p.nv = nv;
  hipError_t e;
  if ((e = hipMalloc(&p.vecs, sizeof(VecDesc) * std::max<int64_t>(nv, 1))) != hipSuccess)
    return hip_fail(e, "lpf_full: plan allocation");
  if ((e = hipMalloc(&p.bin_off, sizeof(int32_t) * off.size())) != hipSuccess)
    return hip_fail(e, "lpf_full: plan allocation");
  if ((e = hipMalloc(&p.dxdy, sizeof(int16_t) * std::max<size_t>(can.size(), 2))) != hipSuccess)
    return hip_fail(e, "lpf_full: plan allocation");
  if ((e = hipMemcpy(p.vecs, vecs.data(), sizeof(VecDesc) * nv, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(p.bin_off, off.data(), sizeof(int32_t) * off.size(), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(p.dxdy, can.data(), sizeof(int16_t) * can.size(), hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e, "lpf_full: plan upload");
  auto res = c->full_plans.emplace(key, p);
  plan = &res.first->second;
  return LPF_OK;
}

int nph_of(unsigned mask) { return (int)(mask & 1u) + (int)((mask >> 1) & 1u); }

}  // namespace

extern "C" {

const char *lpf_last_error(void) { return g_err.c_str(); }

int64_t lpf_num_vectors(int cx, int cy) {
  if (cx < 0 || cy < 0) return -1;
  return (int64_t)(cx + 1) * (cy + 1) + (int64_t)cx * cy;
}

lpf_status lpf_vectors(int cx, int cy, int16_t *dxdy) {
  if (cx < 0 || cy < 0 || cx > 32767 || cy > 32767) return fail(LPF_E_INVAL, "lpf_vectors: cutoff");
  if (!dxdy) return fail(LPF_E_INVAL, "lpf_vectors: dxdy is NULL");
  std::vector<int16_t> v;
  canonical_vectors(cx, cy, v);
  std::memcpy(dxdy, v.data(), v.size() * sizeof(int16_t));
  return LPF_OK;
}

lpf_status lpf_ctx_create(int hip_device, lpf_ctx *out) {
  if (!out) return fail(LPF_E_INVAL, "lpf_ctx_create: out is NULL");
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n)
    return fail(LPF_E_INVAL, "lpf_ctx_create: no such HIP device");
  lpf_ctx c = new (std::nothrow) lpf_ctx_s();
  if (!c) return fail(LPF_E_NOMEM, "lpf_ctx_create: out of host memory");
  c->dev = hip_device;
  DeviceGuard g(c->dev);
  hipError_t e = prepare_full_kernels(kMaxLds);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "lpf_ctx_create: kernel attributes");
  }
  *out = c;
  return LPF_OK;
}

void lpf_ctx_destroy(lpf_ctx c) {
  if (!c) return;
  {
    DeviceGuard g(c->dev);
    (void)hipDeviceSynchronize();
    for (auto &kv : c->full_plans) {
      (void)hipFree(kv.second.vecs);
      (void)hipFree(kv.second.bin_off);
      (void)hipFree(kv.second.dxdy);
    }
    c->ext.release();
    c->part.release();
  }
  delete c;
}

lpf_status lpf_pack(lpf_ctx c, const uint8_t *img, int W, int H, uint64_t *bits, void *stream) {
  if (!c) return fail(LPF_E_INVAL, "lpf_pack: ctx is NULL");
  if (!img || !bits) return fail(LPF_E_INVAL, "lpf_pack: NULL buffer");
  if (W < 1 || H < 1 || W > 65535 || H > 65535) return fail(LPF_E_INVAL, "lpf_pack: W/H out of range");
  DeviceGuard g(c->dev);
  hipError_t e = launch_pack(img, W, H, bits, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "lpf_pack");
  return LPF_OK;
}

lpf_status lpf_full(lpf_ctx c, const uint64_t *bits, int W, int H, int cx, int cy,
                    unsigned phase_mask, int out_layout, uint32_t *counts, void *stream) {
  if (!c) return fail(LPF_E_INVAL, "lpf_full: ctx is NULL");
  if (!bits || !counts) return fail(LPF_E_INVAL, "lpf_full: NULL buffer");
  if (W < 1 || H < 1 || W > 65535 || H > 65535) return fail(LPF_E_INVAL, "lpf_full: W/H out of range");
  if (cx < 0 || cy < 0 || cx > W - 1 || cy > H - 1)
    return fail(LPF_E_INVAL, "lpf_full: cutoff must satisfy 0 <= cx <= W-1, 0 <= cy <= H-1");
  if (phase_mask < 1 || phase_mask > 3) return fail(LPF_E_INVAL, "lpf_full: phase_mask must be 1, 2 or 3");
  if (out_layout != LPF_OUT_HALF && out_layout != LPF_OUT_GRID)
    return fail(LPF_E_INVAL, "lpf_full: out_layout");
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->dev);
  if (!g.ok) return fail(LPF_E_DEVICE, "lpf_full: cannot select the context's device");
  FullPlan *plan = nullptr;
  lpf_status st = get_full_plan(c, W, H, cx, cy, plan);
  if (st != LPF_OK) return st;
  const FullShape &sh = plan->sh;
  const int nph = nph_of(phase_mask);
  const int nv = (int)plan->nv;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if ((e = c->ext.ensure((size_t)H * sh.we * sizeof(uint32_t))) != hipSuccess)
    return hip_fail(e, "lpf_full: scratch");
  const bool direct = sh.ntiles == 1 && out_layout == LPF_OUT_HALF;
  uint32_t *dst = counts;
  if (!direct) {
    if ((e = c->part.ensure((size_t)sh.ntiles * nph * nv * sizeof(uint32_t))) != hipSuccess)
      return hip_fail(e, "lpf_full: scratch");
    dst = (uint32_t *)c->part.p;
  }
  uint32_t *ext = (uint32_t *)c->ext.p;
  if ((e = launch_ext(bits, W, H, sh.we, ext, s)) != hipSuccess) return hip_fail(e, "lpf_full: ext");
  if ((e = launch_full(sh, ext, W, H, cy, plan->vecs, plan->bin_off, phase_mask, dst, nv, s)) != hipSuccess)
    return hip_fail(e, "lpf_full: kernel");
  if (!direct) {
    if ((e = launch_finish(dst, sh.ntiles, nph, nv, plan->dxdy, cx, cy, out_layout, counts, s)) != hipSuccess)
      return hip_fail(e, "lpf_full: finish");
  }
  return LPF_OK;
}

// Tile-shape override used by the autotuner and by tests (0 = automatic choice).
lpf_status lpf_set_full_shape(lpf_ctx c, int R, int S, int waves_per_group, int lds_bytes) {
  if (!c) return fail(LPF_E_INVAL, "lpf_set_full_shape: ctx is NULL");
  auto pow2ok = [](int v, int hi) { return v == 0 || (v >= 1 && v <= hi && (v & (v - 1)) == 0); };
  if (!pow2ok(R, 16) || !pow2ok(S, 64) || waves_per_group < 0 || waves_per_group > 8 ||
      lds_bytes < 0 || lds_bytes > kMaxLds)
    return fail(LPF_E_INVAL, "lpf_set_full_shape: R in {1..16}, S in {1..64} powers of two, "
                             "waves 1..8, lds <= 160 KiB (0 = automatic)");
  std::lock_guard<std::mutex> lk(c->mu);
  c->force_R = R;
  c->force_S = S;
  c->force_wpg = waves_per_group;
  c->force_lds = lds_bytes;
  return LPF_OK;
}

}  // extern "C"
