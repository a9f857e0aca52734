// liblpf C ABI: argument checks, per-context caches and scratch, launch plans.
// Declarations and the contract of every entry point are in include/lpf.h.
#include <algorithm>
#include <cmath>
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

// Fixed device scratch of lpf_full_noalloc: the extended image (H rows of `we` dwords).  Host
// code never passes this name to a kernel or a copy: it stands for a host-side shadow, and the
// device address comes from hipGetSymbolAddress (one per device, taken at context creation).
constexpr size_t kNoAllocWords = (size_t)1 << 20;  // 4 MiB
static __device__ __align__(256) uint32_t scratch[kNoAllocWords];

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

// A buffer that is filled with zeros on stream s when (re)allocated; never called while s is
// being captured.
hipError_t ensure_zeroed(DevBuf &b, size_t n, hipStream_t s) {
  if (n <= b.bytes) return hipSuccess;
  hipError_t e = b.ensure(n);
  if (e == hipSuccess) e = hipMemsetAsync(b.p, 0, n, s);
  return e;
}

struct FullPlan {
  FullShape sh{};
  ChainDesc *chains = nullptr;  // device, bin order
  MemDesc *mems = nullptr;      // device, chain order
  int32_t *bin_off = nullptr;   // device, nbins + 1
  int64_t nv = 0;
  int64_t walk = 0, path_pixels = 0;  // pixels walked per start word; M_c
  std::vector<int64_t> bin_cost;  // host: cost of each bin (pixels + overhead per member)
};

struct TunedShape {
  int R = 0, wpg = 0, lds = 0;
  double ms = 0.0;
};

struct DeltaPlan {
  DeltaGeo geo{};
  DeltaVec *vecs = nullptr;     // device, chunk order
  int32_t *chunk_off = nullptr;  // device, nchunks + 1
  uint32_t *runs = nullptr;      // device run table
  int nchunks = 0;
  int64_t nv = 0;
  bool use_lds = false;
};

// Launch plan of the offset-row delta (plan_delta.hip): vector groups, rows, chunks (device).
// ok = false: the table would exceed kDiagTableMax (the run-based kernel is used instead).
struct DiagPlan {
  DiagGroup *groups = nullptr;
  DiagRow *rows = nullptr;
  int32_t *chunk_off = nullptr;
  int nchunks = 0;
  bool ok = false;
};

// Launch plan of the two-point counts (k_s2.hip).
struct S2Plan {
  int4 *fams = nullptr;      // device: vector families {dx0, dy, members}, sorted by dy
  int4 *groups = nullptr;    // device: {first, end, dy of first, dy of last}
  int32_t *vec = nullptr;    // device, canonical order: (dx & 0xffff) | (dy << 16)
  int ngroups = 0, rb = 0, nrb = 0, we = 0, swd = 0, swdp = 0, J = 1, rstB = 0;
  size_t lds = 0;
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
// staging budget used when an image needs more than the default: leaves room for the batch
// kernel's own LDS word
constexpr int kBigLds = kMaxLds - kBatchStaticLds;

}  // namespace

// Device address of `scratch` per HIP device (filled once per device at context creation).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t *g_scratch_ptr[kMaxDevices] = {};

struct lpf_ctx_s {
  int dev = 0;
  uint32_t *noalloc_scratch = nullptr;  // this device's address of `scratch`
  std::map<std::tuple<int, int, int, int, int, int, int>, FullPlan> full_plans;
  std::map<std::pair<int, int>, ChainSet> chain_sets;  // chains per cutoff (host)
  std::map<std::tuple<int, int, int, int, int>, DeltaPlan> delta_plans;
  std::map<std::tuple<int, int, int>, DiagPlan> diag_plans;  // (cx, cy, chunks)
  std::map<std::tuple<int, int, int, int>, TunedShape> tuned;   // autotuner results
  std::map<std::tuple<int, int, int, int>, S2Plan> s2_plans;
  // 3-D vectors per cutoff, longest first, and the start of each one's voxel-table entries
  struct Vec3 {
    int4 *vec = nullptr;
    int *woff = nullptr;
    int64_t nwalk = 0;  // table entries (int2), a multiple of 2
    // voxel tables per slab geometry (plane stride ps, row stride rst): built once, then only read
    std::map<std::pair<int, int>, int2 *> walk;
  };
  std::map<std::tuple<int, int, int>, Vec3> vec3;
  std::map<std::string, struct BatchGraph *> batch_graphs;
  uint64_t batch_clock = 0;  // use counter of the cached batch graphs
  DevBuf ext, ext3, s2ext, s2acc, sext, rank_buf;
  int s2half = 0;  // lpf_s2: which half of s2acc the next call accumulates into
  std::mutex mu;
  // shape override (autotuner): R, S, wpg, lds budget; 0 = automatic
  int force_R = 0, force_S = 0, force_wpg = 0, force_lds = 0;
  bool force_run_delta = false;  // lpf_delta_swap through the run-based kernel (comparisons)
};


struct lpf_anneal_s {
  lpf_ctx ctx = nullptr;
  bool s2 = false;  // descriptor: two-point probability, else lineal path
  const uint64_t *sample = nullptr;  // Monte-Carlo position set of the cell (caller's), or none
  int64_t Neff = 0;                  // N of the objective: W*H, or the number of sampled positions
  int W = 0, H = 0, cx = 0, cy = 0;
  unsigned mask = 0;
  uint64_t *bits = nullptr;
  uint32_t *counts = nullptr;
  const uint32_t *target = nullptr;
  double *e = nullptr;
  int64_t Nt = 0;
  uint64_t seed = 0;
  AnnealDev *dev = nullptr;  // device struct
  int32_t *pos = nullptr;    // device, W*H: phase-1 list then phase-0 list (reserved in place)
  DevBuf E3, cand, U, slot, S_acc, ksel, dl, ctl;
  bool e3_valid = false;     // E3 holds the current cell (recount method)
  // placement-state records (records method)
  int method = LPF_DELTA_AUTO;
  int rec_choice = -1;  // resolved method (1 records, 0 recount), -1 until first needed
  bool rec_ready = false, rec_valid = false;
  RecGeo rg{};
  DevBuf rmeta, rpix, rvbit, remask, rec, ones, rext, rcond;
  // learned proposals: a network scoring the current cell, or a caller's score field
  lpf_cnn net = nullptr;
  const float *scores_ext = nullptr;
  double beta = 1.0, eps = 0.1;
  int refresh = 1, learn_age = 0;  // learned draws between re-scorings, draws since the last
  bool rank = false;               // evaluate learned draws by descending predicted gain
  DevBuf scores, cw1, cw0, cwb, eS, eCtl, order, rank_buf, S0;
  DevBuf pre;              // uniform draws: the next step's round-0 list slots (ProposeArgs::pre)
  DevBuf Tcur;             // the current step's temperature (device scalar)
  uint64_t host_step = 0;  // host copy of the step counter (steps enqueued so far)
  bool predrawn = false;   // ranked chain: the next step's draws are made by the last step's end
  int predrawn_K = 0;      // ... for that many candidates
  // arguments of those draws per parity of the drawn step, in device memory (nxargs), and the
  // host copies they were made from (nx_ok: uploaded)
  DevBuf nxargs;
  ProposeArgs nx_host[2];
  bool nx_ok[2] = {false, false};
  hipStream_t cap = nullptr;  // private stream for capturing runs of steps
};

// device memory the records method may take by itself (records + ones)
constexpr int64_t kRecBudget = (int64_t)16 << 30;

// A captured lpf_batch launch (extended images, counter reset, persistent kernel).
// Keyed by the descriptors, phase mask, layout and shape overrides, not by the caller's
// buffers: those go through `args`, written before each replay.  At most kMaxBatchGraphs are
// kept; the least recently used is released first.
struct BatchGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  FullImg *imgs = nullptr;
  BatchArgs *args = nullptr;
  int2 *items = nullptr;
  int64_t *bits_off = nullptr, *ext_off = nullptr, *counts_off = nullptr;
  int *counter = nullptr;
  uint32_t *ext = nullptr;
  int n_items = 0, n_wg = 0;
  uint64_t last_use = 0;
};
constexpr size_t kMaxBatchGraphs = 16;

struct lpf_cnn_s {
  lpf_ctx ctx = nullptr;
  int W = 0, H = 0, max_batch = 0, max_samples = 0;
  CnnBufs b{};
  std::vector<void *> allocs;
};

namespace {

void free_batch_graph(BatchGraph *b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  (void)hipFree(b->imgs);
  (void)hipFree(b->args);
  (void)hipFree(b->items);
  (void)hipFree(b->bits_off);
  (void)hipFree(b->ext_off);
  (void)hipFree(b->counts_off);
  (void)hipFree(b->counter);
  (void)hipFree(b->ext);
  delete b;
}

void release_batch_graphs(lpf_ctx c);

bool choose_shape(lpf_ctx c, int W, int H, int cx, int cy, FullShape &sh, std::string &why) {
  const int swd = (W + 31) / 32;
  const TunedShape *tuned = nullptr;
  auto tk = c->tuned.find(std::make_tuple(W, H, cx, cy));
  if (tk != c->tuned.end()) tuned = &tk->second;
  int fR = c->force_R ? c->force_R : (tuned ? tuned->R : 0);
  int fW = c->force_wpg ? c->force_wpg : (tuned ? tuned->wpg : 0);
  int fL = c->force_lds ? c->force_lds : (tuned ? tuned->lds : 0);
  // up to 16 words per lane (the autotuner's choice at W = 128, 256, 512 and 1024)
  int R = fR ? fR : std::min(16, next_pow2(swd));
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
  // 8 waves per group when one tile fits the default budget (two groups per CU), else 16 (below)
  sh.wpg = fW ? fW : 8;
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
  int budget = fL ? fL : 64 * 1024;
  sh.glob = 0;
  for (;;) {
    int tile;
    const int slots = kSlotWords * 4;  // count slots of the bin's members
    const int rows_max = (budget - slots) / (sh.rst * 4);
    if (rows_max - cy - rpw >= H) {
      tile = H;
    } else {
      tile = ((rows_max - cy - rpw) / rpw) * rpw;
    }
    if (tile >= 1) {
      sh.tile = tile;
      break;
    }
    if (budget >= kBigLds || fL) {
      // the halo rows do not fit in the staging budget: read the rows of the periodically
      // extended image from device memory (L2) instead, one tile of all H rows
      sh.glob = 1;
      sh.tile = H;
      sh.rst = sh.we;
      break;
    }
    budget = kBigLds;
    // one workgroup per CU at this budget: 16 waves keep four per SIMD (1 024² at cutoff 512:
    // 199 ms against 244 ms with 8)
    if (!fW) sh.wpg = 16;
  }
  sh.ntiles = (H + sh.tile - 1) / sh.tile;
  sh.lds_rows = sh.tile + cy + rpw;
  // waves sharing a chain: as many as the tile has bands (a power of two dividing wpg)
  const int bands = (sh.tile + rpw - 1) / rpw;
  sh.nwb = 1;
  while (sh.nwb * 2 <= std::min(sh.wpg, bands) && sh.wpg % (sh.nwb * 2) == 0) sh.nwb *= 2;
  return true;
}

lpf_status get_full_plan(lpf_ctx c, int W, int H, int cx, int cy, FullPlan *&plan) {
  FullShape sh{};
  std::string why;
  if (!choose_shape(c, W, H, cx, cy, sh, why)) return fail(LPF_E_UNSUPPORTED, "lpf_full: " + why);
  if (full_lds_bytes(sh, sh.wpg) > (size_t)kMaxLds)
    return fail(LPF_E_UNSUPPORTED, "lpf_full: tile shape needs more than 160 KiB of LDS");
  auto key = std::make_tuple(W, H, cx, cy, sh.R * 1000 + sh.S, sh.wpg, 2 * sh.tile + sh.glob);
  auto it = c->full_plans.find(key);
  if (it != c->full_plans.end()) {
    plan = &it->second;
    return LPF_OK;
  }
  const int64_t nv = lpf_num_vectors(cx, cy);
  if (nv > (int64_t)1 << 30) return fail(LPF_E_UNSUPPORTED, "lpf_full: too many vectors");
  auto chs = c->chain_sets.find(std::make_pair(cx, cy));
  if (chs == c->chain_sets.end()) {
    build_chains(cx, cy, c->chain_sets[std::make_pair(cx, cy)]);
    chs = c->chain_sets.find(std::make_pair(cx, cy));
  }
  const ChainSet &all = chs->second;
  // Workgroup-level bins of chain pieces (pack_bins): twice as many bins as the device holds
  // workgroups at once (each walks about the same number of pixels; the second wave of
  // workgroups evens out what the cost model misses), fewer when there are too few chains to
  // keep each wave of a workgroup busy.
  const int nwc = sh.wpg / sh.nwb;
  int cus = 256;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->dev);
  const int resident = cus * full_wgs_per_cu(sh.R, false, sh.wpg, full_lds_bytes(sh, sh.wpg));
  const int64_t nb_want =
      std::min<int64_t>(2 * resident, std::max<int64_t>(1, (int64_t)all.chains.size() / (4 * nwc)));
  BinPlan bp;
  pack_bins(all, nb_want, bp);
  sh.nbins = bp.nbins;
  const std::vector<ChainDesc> &chains = bp.chains;
  const std::vector<MemDesc> &mems = bp.mems;
  const std::vector<int32_t> &off = bp.off;

  FullPlan p;
  p.sh = sh;
  p.nv = nv;
  p.walk = all.walk;
  p.path_pixels = all.path_pixels;
  hipError_t e;
  if ((e = hipMalloc(&p.chains, sizeof(ChainDesc) * std::max<size_t>(chains.size(), 1))) != hipSuccess ||
      (e = hipMalloc(&p.mems, sizeof(MemDesc) * std::max<size_t>(mems.size(), 1))) != hipSuccess ||
      (e = hipMalloc(&p.bin_off, sizeof(int32_t) * off.size())) != hipSuccess) {
    (void)hipFree(p.chains);
    (void)hipFree(p.mems);
    return hip_fail(e, "lpf_full: plan allocation");
  }
  if ((e = hipMemcpy(p.chains, chains.data(), sizeof(ChainDesc) * chains.size(), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(p.mems, mems.data(), sizeof(MemDesc) * mems.size(), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(p.bin_off, off.data(), sizeof(int32_t) * off.size(), hipMemcpyHostToDevice)) != hipSuccess) {
    (void)hipFree(p.chains);
    (void)hipFree(p.mems);
    (void)hipFree(p.bin_off);
    return hip_fail(e, "lpf_full: plan upload");
  }
  p.bin_cost = bp.cost;
  auto res = c->full_plans.emplace(key, p);
  plan = &res.first->second;
  return LPF_OK;
}

void release_batch_graphs(lpf_ctx c) {
  for (auto &kv : c->batch_graphs) free_batch_graph(kv.second);
  c->batch_graphs.clear();
}

// Two-point counts plan.  Vector families {dx0, dy, nj}: for each dy, the dx of D_c taken in
// 32 residue classes, each class cut into runs of at most J members 32 apart (J = 1, 2, 4 or 8
// from the widest dx range); families sorted by dy and cut into groups of at most 64 (one per
// lane; the four waves of a workgroup share them) whose dy range keeps the staged rows within
// the LDS budget; start rows in blocks of rb (32, halved down to 8 while the launch has fewer
// than about 1024 workgroups).
lpf_status get_s2_plan(lpf_ctx c, int W, int H, int cx, int cy, S2Plan *&plan) {
  auto key = std::make_tuple(W, H, cx, cy);
  auto it = c->s2_plans.find(key);
  if (it != c->s2_plans.end()) {
    plan = &it->second;
    return LPF_OK;
  }
  const int64_t nv = lpf_num_vectors(cx, cy);
  if (nv > (int64_t)1 << 30) return fail(LPF_E_UNSUPPORTED, "lpf_s2: too many vectors");
  S2Plan p;
  const int range = cy > 0 ? 2 * cx + 1 : cx + 1;  // widest dx range of one dy
  p.J = std::min(8, next_pow2((range + 31) / 32));
  p.swd = (W + 31) / 32;
  p.swdp = (p.swd + 7) / 8 * 8;
  p.we = ((W + cx) >> 5) + p.swdp + p.J;  // the last gather of a family: (s0 >> 5) + swdp + J - 1
  p.rstB = p.we | 1;
  // rows A and B, then the cross-wave reduction (4 waves x J members x 64 lanes)
  auto bytes = [&](int rb, int span) {
    return ((size_t)rb * p.swdp + (size_t)(rb + span) * p.rstB + (size_t)4 * p.J * 64) *
           sizeof(uint32_t);
  };
  size_t budget = 64 * 1024;
  // blocks of 16 start rows (512^2, cutoff 128: 2 144 workgroups, 0.031 ms per call against
  // 0.033 with 32 or 64 rows and 0.032 with 8; the span rows staged per block weigh less than
  // the launch's tail)
  int rb = std::min(16, H);
  while (rb > 1 && 2 * bytes(rb, 0) > budget) rb = (rb + 1) / 2;
  if (bytes(rb, 0) > budget) budget = kMaxLds;
  if (bytes(rb, 0) > budget) return fail(LPF_E_UNSUPPORTED, "lpf_s2: rows too wide for LDS staging");
  const int span_max = (int)((budget / 4 - (size_t)rb * p.swdp - (size_t)4 * p.J * 64) / p.rstB) - rb;
  std::vector<int4> fams;
  for (int dy = 0; dy <= cy; ++dy) {
    const int lo = dy == 0 ? 0 : -cx;
    const int n = dy == 0 ? cx + 1 : 2 * cx + 1;
    for (int r = 0; r < std::min(32, n); ++r) {
      const int members = (n - r + 31) / 32;
      for (int m = 0; m < members; m += p.J)
        fams.push_back(make_int4(lo + r + 32 * m, dy, std::min(p.J, members - m), 0));
    }
  }
  std::vector<int4> groups;
  int max_span = 0;
  const int64_t nf = (int64_t)fams.size();
  for (int64_t i = 0; i < nf;) {
    int64_t j = i;
    const int dy0 = fams[i].y;
    while (j < nf && j - i < 64 && fams[j].y - dy0 <= span_max) ++j;
    groups.push_back(make_int4((int)i, (int)j, dy0, fams[j - 1].y));
    max_span = std::max(max_span, fams[j - 1].y - dy0);
    i = j;
  }
  while (rb > 8 && (int64_t)groups.size() * ((H + rb - 1) / rb) < 1024) rb /= 2;
  std::vector<int32_t> packed(nv);
  {
    std::vector<int16_t> can;
    canonical_vectors(cx, cy, can);
    for (int64_t i = 0; i < nv; ++i)
      packed[i] = (int32_t)((uint32_t)(uint16_t)can[2 * i] | ((uint32_t)(uint16_t)can[2 * i + 1] << 16));
  }
  p.rb = rb;
  p.nrb = (H + rb - 1) / rb;
  p.ngroups = (int)groups.size();
  p.lds = bytes(rb, max_span);
  p.nv = nv;
  hipError_t e;
  if ((e = hipMalloc(&p.fams, sizeof(int4) * fams.size())) != hipSuccess ||
      (e = hipMalloc(&p.groups, sizeof(int4) * groups.size())) != hipSuccess ||
      (e = hipMalloc(&p.vec, sizeof(int32_t) * nv)) != hipSuccess) {
    (void)hipFree(p.fams);
    (void)hipFree(p.groups);
    (void)hipFree(p.vec);
    return hip_fail(e, "lpf_s2: plan allocation");
  }
  if ((e = hipMemcpy(p.fams, fams.data(), sizeof(int4) * fams.size(), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(p.groups, groups.data(), sizeof(int4) * groups.size(), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(p.vec, packed.data(), sizeof(int32_t) * nv, hipMemcpyHostToDevice)) != hipSuccess) {
    (void)hipFree(p.fams);
    (void)hipFree(p.groups);
    (void)hipFree(p.vec);
    return hip_fail(e, "lpf_s2: plan upload");
  }
  auto res = c->s2_plans.emplace(key, p);
  plan = &res.first->second;
  return LPF_OK;
}

// Rounds of an S2 chain: candidates per workgroup and vector chunks (enough workgroups to fill
// the device, at least 8 vectors per thread).
void s2_rounds(std::vector<RoundPlan> &rounds, int64_t nv) {
  for (RoundPlan &r : rounds) {
    r.block = r.C <= 64 ? 64 : (r.C <= 128 ? 128 : 256);
    const int groups = (r.C + r.block - 1) / r.block;
    r.nchunks = (int)std::max<int64_t>(1, std::min<int64_t>(2048 / groups, nv / 8));
  }
}

// The packed cell fits the S2 round kernel's LDS staging.
bool s2_img_lds(int W, int H) { return (size_t)H * ((W + 63) / 64) * 8 <= 64 * 1024; }

int nph_of(unsigned mask) { return (int)(mask & 1u) + (int)((mask >> 1) & 1u); }

FullImg make_img(const FullPlan &p, const uint32_t *ext, uint32_t *out, int W, int H, int cx,
                 int cy, int layout) {
  FullImg I{};
  I.E = ext;
  I.out = out;
  I.chains = p.chains;
  I.mems = p.mems;
  I.bin_off = p.bin_off;
  I.nwb = p.sh.nwb;
  I.glob = p.sh.glob;
  I.W = W;
  I.H = H;
  I.cx = cx;
  I.cy = cy;
  I.R = p.sh.R;
  I.S = p.sh.S;
  I.we = p.sh.we;
  I.rst = p.sh.rst;
  I.tile = p.sh.tile;
  I.ntiles = p.sh.ntiles;
  I.lds_rows = p.sh.lds_rows;
  I.nv = (int)p.nv;
  I.layout = layout;
  I.nbins = p.sh.nbins;
  return I;
}

// delta-kernel staging of the three image frames (below 64 KiB, the kernels' static words aside)
constexpr int kDeltaLdsMax = 60 * 1024;

// Geometry of the three frames used by the delta kernel (image, transposed, anti-transposed).
DeltaGeo delta_geometry(int W, int H, int cx, int cy) {
  DeltaGeo g{};
  g.hy = std::min(cx, cy);
  const int dims[3][3] = {{W, H, cx}, {H, W, cy}, {H, W, cy}};  // width, height, max major extent
  int off = 0;
  for (int i = 0; i < 3; ++i) {
    ImgGeo &im = g.g[i];
    im.W = dims[i][0];
    im.H = dims[i][1];
    im.we = ((im.W - 1 + dims[i][2]) >> 5) + 3;
    im.off = off;
    uint64_t pat = 0;
    for (int t = 0; t < 64; t += im.W) pat |= 1ull << t;
    im.pat = pat;
    off += (im.H + g.hy) * im.we;
  }
  g.total = off;
  return g;
}

lpf_status get_delta_plan(lpf_ctx c, int W, int H, int cx, int cy, int nchunks_req,
                          DeltaPlan *&plan) {
  std::vector<int16_t> can;
  canonical_vectors(cx, cy, can);
  const int64_t nv = (int64_t)can.size() / 2;
  const int nchunks = (int)std::max<int64_t>(1, std::min<int64_t>(nchunks_req, nv));
  auto key = std::make_tuple(W, H, cx, cy, nchunks);
  auto it = c->delta_plans.find(key);
  if (it != c->delta_plans.end()) {
    plan = &it->second;
    return LPF_OK;
  }
  // Flat form of every vector: frame, major extent n, minor extent m, mirrored in x or not.
  std::vector<DeltaVec> dv(nv);
  std::vector<uint32_t> runs;
  std::vector<int64_t> cost(nv);
  for (int64_t i = 0; i < nv; ++i) {
    const int dx = can[2 * i], dy = can[2 * i + 1];
    const int adx = std::abs(dx);
    int img, n, m;
    bool q2;
    if (adx >= dy) {
      img = 0; n = adx; m = dy; q2 = dx < 0;
    } else if (dx >= 0) {
      img = 1; n = dy; m = dx; q2 = false;
    } else {
      img = 2; n = dy; m = adx; q2 = true;
    }
    // runs of the digitised flat segment: row j holds x with floor((2xm + n) / (2n)) == j
    std::vector<int> lo(m + 1, -1), hi(m + 1, -1);
    for (int x = 0; x <= n; ++x) {
      const int j = n ? (int)((2LL * x * m + n) / (2LL * n)) : 0;
      if (lo[j] < 0) lo[j] = x;
      hi[j] = x;
    }
    dv[i] = DeltaVec{m, (int32_t)i, img, (int32_t)runs.size()};
    int64_t px_tot = 0;
    for (int j = 0; j <= m; ++j) {
      const int a = q2 ? n - hi[j] : lo[j];
      const int b = q2 ? n - lo[j] : hi[j];
      runs.push_back((uint32_t)a | ((uint32_t)b << 16));
      px_tot += (b - a) / 32 + 1;
    }
    cost[i] = (int64_t)(m + 1) * (4 * (n + 1) + 15 * (m + 1) * 1 + 15 * px_tot) + 8;
  }
  // chunks: longest-processing-time-first
  std::vector<int> order(nv);
  for (int64_t i = 0; i < nv; ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  using Item = std::pair<int64_t, int>;
  std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
  for (int b = 0; b < nchunks; ++b) heap.push({0, b});
  std::vector<std::vector<int>> bins(nchunks);
  for (int i : order) {
    Item t = heap.top();
    heap.pop();
    bins[t.second].push_back(i);
    heap.push({t.first + cost[i], t.second});
  }
  std::vector<DeltaVec> vs;
  vs.reserve(nv);
  std::vector<int32_t> off(nchunks + 1, 0);
  for (int b = 0; b < nchunks; ++b) {
    off[b] = (int32_t)vs.size();
    for (int i : bins[b]) vs.push_back(dv[i]);
  }
  off[nchunks] = (int32_t)vs.size();
  DeltaPlan p;
  p.geo = delta_geometry(W, H, cx, cy);
  p.nchunks = nchunks;
  p.nv = nv;
  p.use_lds = (int64_t)p.geo.total * 4 <= kDeltaLdsMax;
  hipError_t e;
  if ((e = hipMalloc(&p.vecs, sizeof(DeltaVec) * vs.size())) != hipSuccess ||
      (e = hipMalloc(&p.chunk_off, sizeof(int32_t) * off.size())) != hipSuccess ||
      (e = hipMalloc(&p.runs, sizeof(uint32_t) * runs.size())) != hipSuccess)
    return hip_fail(e, "delta plan allocation");
  if ((e = hipMemcpy(p.vecs, vs.data(), sizeof(DeltaVec) * vs.size(), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(p.chunk_off, off.data(), sizeof(int32_t) * off.size(), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(p.runs, runs.data(), sizeof(uint32_t) * runs.size(), hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e, "delta plan upload");
  auto res = c->delta_plans.emplace(key, p);
  plan = &res.first->second;
  return LPF_OK;
}

constexpr size_t kDiagTableMax = (size_t)256 << 20;  // bytes of offset rows per plan

lpf_status get_diag_plan(lpf_ctx c, int cx, int cy, int nchunks_req, DiagPlan *&plan) {
  auto key = std::make_tuple(cx, cy, nchunks_req);
  auto it = c->diag_plans.find(key);
  if (it != c->diag_plans.end()) {
    plan = &it->second;
    return LPF_OK;
  }
  DiagPlan p;
  DiagTable t;
  bool built = false;
  try {
    built = std::max(cx, cy) <= 255 && build_diag_table(cx, cy, nchunks_req, kDiagTableMax, t);
  } catch (const std::exception &ex) {
    return fail(LPF_E_UNSUPPORTED, std::string("delta table: ") + ex.what());
  }
  if (built) {
    hipError_t e;
    if ((e = hipMalloc(&p.groups, sizeof(DiagGroup) * t.groups.size())) != hipSuccess ||
        (e = hipMalloc(&p.rows, sizeof(DiagRow) * std::max<size_t>(1, t.rows.size()))) != hipSuccess ||
        (e = hipMalloc(&p.chunk_off, sizeof(int32_t) * t.chunk_off.size())) != hipSuccess) {
      (void)hipFree(p.groups);
      (void)hipFree(p.rows);
      (void)hipFree(p.chunk_off);
      return hip_fail(e, "delta table allocation");
    }
    if ((e = hipMemcpy(p.groups, t.groups.data(), sizeof(DiagGroup) * t.groups.size(), hipMemcpyHostToDevice)) != hipSuccess ||
        (!t.rows.empty() && (e = hipMemcpy(p.rows, t.rows.data(), sizeof(DiagRow) * t.rows.size(), hipMemcpyHostToDevice)) != hipSuccess) ||
        (e = hipMemcpy(p.chunk_off, t.chunk_off.data(), sizeof(int32_t) * t.chunk_off.size(), hipMemcpyHostToDevice)) != hipSuccess) {
      (void)hipFree(p.groups);
      (void)hipFree(p.rows);
      (void)hipFree(p.chunk_off);
      return hip_fail(e, "delta table upload");
    }
    p.nchunks = (int)t.chunk_off.size() - 1;
    p.ok = true;
  }
  auto res = c->diag_plans.emplace(key, p);
  plan = &res.first->second;
  return LPF_OK;
}

// Number of vector chunks for K candidates: enough workgroups to fill the device.
int delta_chunks(int K) {
  const int groups = (K + 255) / 256;
  return std::max(1, 2048 / groups);
}

// Candidates of the chain's current step into a->cand / U / slot (learned weights first), in the
// half of those double-buffered arrays that the step's parity selects; with rank, learned draws
// also leave their rank keys and workgroup lists in a->rank_buf.  With defer, the draws'
// arguments go to *defer for a launch that also evaluates round 0 (or for none: the previous
// step's end made them), and nothing but the learned weights is launched here.  args: when
// given, also receives the arguments.  upkeep false: the learned proposal's re-scoring and draw
// count are left alone (a draw made ahead of its step).
lpf_status draw_candidates(lpf_anneal a, int K, int proposal, hipStream_t s,
                           int64_t *S_acc = nullptr, StepCtl *ctl = nullptr,
                           const double *T_sched = nullptr, int64_t T_base = 0, double T = 0.0,
                           double *T_cur = nullptr, bool rank = false,
                           ProposeArgs *defer = nullptr, ProposeArgs *args = nullptr,
                           bool upkeep = true) {
  hipError_t e;
  const int64_t N = (int64_t)a->W * a->H;
  if ((e = a->cand.ensure(sizeof(int2) * 2 * (size_t)K)) != hipSuccess ||
      (e = a->U.ensure(sizeof(double) * 2 * (size_t)K)) != hipSuccess ||
      (e = a->slot.ensure(sizeof(int2) * 2 * (size_t)K)) != hipSuccess)
    return hip_fail(e, "anneal: candidate scratch");
  const size_t half = (size_t)(a->host_step & 1) * (size_t)K;
  const double *cw1 = nullptr, *cw0 = nullptr;
  const float *rank_score = nullptr;
  uint64_t *rank_keys = nullptr;
  int draw = proposal;
  if (proposal == LPF_PROP_LEARNED) {
    // beta = 0 draws exactly the uniform candidates; the scores then only rank them
    const bool weighted = a->beta > 0.0;
    if (weighted && ((e = a->cw1.ensure(sizeof(double) * (size_t)N)) != hipSuccess ||
                     (e = a->cw0.ensure(sizeof(double) * (size_t)N)) != hipSuccess ||
                     (e = a->cwb.ensure(sizeof(double) * 4 * (size_t)((N + 1023) / 1024))) != hipSuccess))
      return hip_fail(e, "anneal: proposal scratch");
    if (upkeep && (a->learn_age == 0 || a->learn_age >= a->refresh)) {
      const float *sc = a->scores_ext;
      if (a->net) {
        if ((e = a->scores.ensure(sizeof(float) * (size_t)N)) != hipSuccess)
          return hip_fail(e, "anneal: score scratch");
        if ((e = cnn_score(a->net->b, a->bits, a->W, a->H, (float *)a->scores.p, s)) != hipSuccess)
          return hip_fail(e, "anneal: proposal network");
        sc = (const float *)a->scores.p;
      }
      if (weighted &&
          (e = launch_learn_weights(a->dev, sc, a->beta, (double *)a->cw1.p, (double *)a->cw0.p, N,
                                    (double *)a->cwb.p, s)) != hipSuccess)
        return hip_fail(e, "anneal: proposal weights");
      a->learn_age = 0;
    }
    if (upkeep) ++a->learn_age;
    if (weighted) {
      cw1 = (const double *)a->cw1.p;
      cw0 = (const double *)a->cw0.p;
    } else {
      draw = LPF_PROP_UNIFORM;
    }
    if (rank) {
      if ((e = a->rank_buf.ensure(kRankScratch)) != hipSuccess)
        return hip_fail(e, "anneal: rank scratch");
      rank_score = a->net ? (const float *)a->scores.p : a->scores_ext;
      rank_keys = (uint64_t *)a->rank_buf.p;
    }
  }
  ProposeArgs p;
  p.st = a->dev;
  p.bits = a->bits;
  p.W = a->W;
  p.H = a->H;
  p.seed = a->seed;
  p.K = K;
  p.proposal = draw;
  p.cw1 = cw1;
  p.cw0 = cw0;
  p.eps = a->eps;
  p.cand = (int2 *)a->cand.p + half;
  p.U = (double *)a->U.p + half;
  p.slot = (int2 *)a->slot.p + half;
  p.S_acc = S_acc;
  p.ctl = ctl;
  p.T_sched = T_sched;
  p.T_base = T_base;
  p.T = T;
  p.T_cur = T_cur;
  p.rank_score = rank_score;
  p.rank_keys = rank_keys;
  p.rank_lists = rank_keys ? rank_keys + kRankMax : nullptr;
  // a round 0 drawn in its own launch reads the slots the previous step's draw wrote
  p.pre = defer && !rank && draw == LPF_PROP_UNIFORM && a->pre.p ? (int4 *)a->pre.p : nullptr;
  if (args) *args = p;
  if (defer) {
    *defer = p;
    return LPF_OK;
  }
  if ((e = launch_propose(p, s)) != hipSuccess)
    return hip_fail(e, "anneal: propose");
  return LPF_OK;
}

// The arguments of a ranked step's draws made by the previous step's end, drawing into half h
// of the candidate buffers (from the step's own arguments; no resets).
ProposeArgs next_args_of(const ProposeArgs &p, lpf_anneal a, int K, int h) {
  ProposeArgs q = p;
  q.cand = (int2 *)a->cand.p + (size_t)h * K;
  q.slot = (int2 *)a->slot.p + (size_t)h * K;
  q.U = (double *)a->U.p + (size_t)h * K;
  q.S_acc = nullptr;
  q.ctl = nullptr;
  q.T_cur = nullptr;
  q.pre = nullptr;
  q.T_sched = nullptr;
  q.T_base = 0;
  q.T = 0.0;
  return q;
}

bool same_next_args(const ProposeArgs &x, const ProposeArgs &y) {
  return x.st == y.st && x.bits == y.bits && x.W == y.W && x.H == y.H && x.seed == y.seed &&
         x.K == y.K && x.proposal == y.proposal && x.cw1 == y.cw1 && x.cw0 == y.cw0 &&
         x.eps == y.eps && x.cand == y.cand && x.U == y.U && x.slot == y.slot &&
         x.rank_score == y.rank_score && x.rank_keys == y.rank_keys &&
         x.rank_lists == y.rank_lists;
}

// Candidate rounds of a step: 64, then the rest in rounds of at most 8192.  A step whose first
// candidates are accepted costs one small round; a skipped round costs two empty launches.
std::vector<RoundPlan> step_rounds(int K, bool decide) {
  std::vector<RoundPlan> r;
  int k0 = 0;
  while (k0 < K) {
    int C = decide ? (k0 == 0 ? 64 : 8192) : 8192;
    C = std::min(std::min(C, 8192), K - k0);
    RoundPlan p{};
    p.k0 = k0;
    p.C = C;
    r.push_back(p);
    k0 += C;
  }
  return r;
}

// Memory the records method needs, and whether it applies at all.
bool records_fit(lpf_anneal a, int64_t *bytes, std::string *why) {
  const int64_t N = (int64_t)a->W * a->H;
  const int64_t nv = lpf_num_vectors(a->cx, a->cy);
  const int nph = nph_of(a->mask);
  int64_t Mc = 0;
  {
    std::vector<int16_t> can;
    canonical_vectors(a->cx, a->cy, can);
    for (int64_t i = 0; i < nv; ++i) Mc += std::max(std::abs((int)can[2 * i]), (int)can[2 * i + 1]) + 1;
  }
  const int64_t Rw = (Mc + 31) / 32 + 2;  // two padding words per plane
  // records, ones, and the build's condition rows
  const int64_t b = N * 2 * nph * Rw * 4 + nv * ((int64_t)((a->W + 7) / 8) * ((a->H + 7) / 8) * 64) +
                    nv * 2 * nph * (int64_t)a->H * ((a->W - 1) / 32 + 3) * 4;
  if (bytes) *bytes = b;
  if (std::max(a->cx, a->cy) > 254) {
    if (why) *why = "cutoff above 254 (path counts are bytes)";
    return false;
  }
  if ((N + 255) / 256 > 65535 || nv > 65535LL * 256) {
    if (why) *why = "image too large for the records kernels";
    return false;
  }
  return true;
}

bool use_records(lpf_anneal a) {
  if (a->rec_choice >= 0) return a->rec_choice == 1;
  if (a->sample) {  // only the records carry a position set (checked at creation)
    a->rec_choice = 1;
    return true;
  }
  int64_t bytes = 0;
  bool rec;
  if (a->method == LPF_DELTA_RECOUNT || !records_fit(a, &bytes, nullptr)) {
    rec = false;
  } else if (a->method == LPF_DELTA_RECORDS) {
    rec = true;
  } else {
    size_t free_b = 0, total_b = 0;
    rec = hipMemGetInfo(&free_b, &total_b) == hipSuccess && bytes <= kRecBudget &&
          bytes <= (int64_t)(free_b / 2);
  }
  a->rec_choice = rec ? 1 : 0;
  return rec;
}

// Host tables and device buffers of the records method; records built from the current cell
// when they are not valid.
lpf_status setup_records(lpf_anneal a, hipStream_t s) {
  hipError_t e;
  if (!a->rec_ready) {
    std::vector<int16_t> can;
    canonical_vectors(a->cx, a->cy, can);
    const int64_t nv = (int64_t)can.size() / 2;
    std::vector<int4> meta(nv);
    std::vector<int32_t> pix, vbit;
    for (int64_t i = 0; i < nv; ++i) {
      const int dx = can[2 * i], dy = can[2 * i + 1];
      const int adx = std::abs(dx), n = std::max(adx, dy);
      meta[i] = make_int4((int)pix.size(), n, dx, dy);
      // the digitised segment (Sec. 2.2), minor coordinate sgn(m) floor((2k|m| + n) / (2n))
      for (int k = 0; k <= n; ++k) {
        int px, py;
        if (adx >= dy) {
          px = dx >= 0 ? k : -k;
          py = n ? (int)((2LL * k * dy + n) / (2LL * n)) : 0;
        } else {
          py = k;
          const int g = (int)((2LL * k * adx + n) / (2LL * n));
          px = dx >= 0 ? g : -g;
        }
        pix.push_back((int32_t)((uint32_t)(uint16_t)(int16_t)px | ((uint32_t)py << 16)));
        vbit.push_back((int32_t)((i << 8) | n));
      }
    }
    // error-term masks of the paths of fewer than 64 pixels (RecGeo::emask): per threshold t
    // from 2n down to 0, the indices whose error term is at least t
    std::vector<uint64_t> emask(2 * pix.size() - (size_t)nv, 0ull);
    for (int64_t i = 0; i < nv; ++i) {
      const int off = meta[i].x, n = meta[i].y, adx = std::abs(meta[i].z), dy = meta[i].w;
      if (n == 0 || n + 1 > 64) continue;
      const int ext = adx >= dy ? dy : adx, n2 = 2 * n;
      std::vector<uint64_t> eq((size_t)n2, 0ull);
      for (int k = 0; k <= n; ++k) eq[(size_t)((2LL * k * ext + n) % n2)] |= 1ull << k;
      const size_t b0 = (size_t)(2 * (int64_t)off - i);
      for (int t = n2 - 1; t >= 0; --t) emask[b0 + t] = emask[b0 + t + 1] | eq[(size_t)t];
    }
    RecGeo g{};
    g.nv = (int)nv;
    g.Mc = (int)pix.size();
    g.Rw = (g.Mc + 31) / 32 + 2;  // two padding words: ranges read three words at once
    g.nph = nph_of(a->mask);
    g.W = a->W;
    g.H = a->H;
    g.rstride = (int64_t)2 * g.nph * g.Rw;
    g.oplane = (int64_t)((a->W + 7) / 8) * ((a->H + 7) / 8) * 64;
    g.mask = a->mask;
    g.sample = a->sample;
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, a->ctx->dev);
    g.end_wgs = rec_end_workgroups(g, cus);
    g.ew = (a->W + 31) / 32 + 2;
    g.cw = (a->W - 1) / 32 + 3;
    const int64_t N = (int64_t)a->W * a->H;
    if ((e = a->rmeta.ensure(sizeof(int4) * meta.size())) != hipSuccess ||
        (e = a->rpix.ensure(sizeof(int32_t) * pix.size())) != hipSuccess ||
        (e = a->rvbit.ensure(sizeof(int32_t) * vbit.size())) != hipSuccess ||
        (e = a->remask.ensure(sizeof(uint64_t) * emask.size())) != hipSuccess ||
        (e = a->rext.ensure(sizeof(uint32_t) * (size_t)g.H * g.ew * (a->sample ? 2 : 1))) != hipSuccess ||
        (e = a->rcond.ensure(sizeof(uint32_t) * (size_t)nv * 2 * g.nph * g.H * g.cw)) != hipSuccess ||
        (e = a->rec.ensure(sizeof(uint32_t) * (size_t)(N * g.rstride))) != hipSuccess ||
        (e = a->ones.ensure((size_t)(nv * g.oplane))) != hipSuccess)
      return hip_fail(e, "anneal: records allocation");
    if ((e = hipMemcpyAsync(a->rmeta.p, meta.data(), sizeof(int4) * meta.size(), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(a->rpix.p, pix.data(), sizeof(int32_t) * pix.size(), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(a->rvbit.p, vbit.data(), sizeof(int32_t) * vbit.size(), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(a->remask.p, emask.data(), sizeof(uint64_t) * emask.size(), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
      return hip_fail(e, "anneal: records tables");
    g.meta = (const int4 *)a->rmeta.p;
    g.pix = (const int32_t *)a->rpix.p;
    g.vbit = (const int32_t *)a->rvbit.p;
    g.emask = (const uint64_t *)a->remask.p;
    g.ext = (uint32_t *)a->rext.p;
    g.cond = (uint32_t *)a->rcond.p;
    g.rec = (uint32_t *)a->rec.p;
    g.ones = (uint8_t *)a->ones.p;
    a->rg = g;
    a->rec_ready = true;
  }
  if (!a->rec_valid) {
    if ((e = launch_rec_build(a->rg, a->bits, s)) != hipSuccess) return hip_fail(e, "anneal: records");
    a->rec_valid = true;
  }
  return LPF_OK;
}

// Round plans of the recount method: candidates per workgroup and vector chunks per round.
lpf_status recount_rounds(lpf_anneal a, std::vector<RoundPlan> &rounds, DeltaPlan *&any) {
  for (RoundPlan &r : rounds) {
    r.block = r.C <= 64 ? 64 : (r.C <= 128 ? 128 : 256);
    const int groups = (r.C + r.block - 1) / r.block;
    DeltaPlan *plan = nullptr;
    lpf_status st = get_delta_plan(a->ctx, a->W, a->H, a->cx, a->cy, std::max(1, 2048 / groups), plan);
    if (st != LPF_OK) return st;
    r.vecs = plan->vecs;
    r.chunk_off = plan->chunk_off;
    r.nchunks = plan->nchunks;
    any = plan;
  }
  return LPF_OK;
}

void records_rounds(std::vector<RoundPlan> &rounds) {
  for (RoundPlan &r : rounds) r.block = 256;
}

// The evaluation state of the chosen method: records, or the three image frames.
lpf_status prepare_eval(lpf_anneal a, bool rec, const DeltaGeo &geo, hipStream_t s) {
  if (rec) return setup_records(a, s);
  hipError_t e;
  if ((e = a->E3.ensure((size_t)geo.total * 4)) != hipSuccess) return hip_fail(e, "anneal: frames");
  if (!a->e3_valid) {
    if ((e = launch_ext3(a->bits, a->W, a->H, geo, (uint32_t *)a->E3.p, s)) != hipSuccess)
      return hip_fail(e, "anneal: frames");
    a->e3_valid = true;
  }
  return LPF_OK;
}

lpf_status check_image_args(const char *fn, int W, int H, int cx, int cy, unsigned mask) {
  if (W < 1 || H < 1 || W > 65535 || H > 65535)
    return fail(LPF_E_INVAL, std::string(fn) + ": W/H out of range");
  if (cx < 0 || cy < 0 || cx > W - 1 || cy > H - 1)
    return fail(LPF_E_INVAL, std::string(fn) + ": cutoff must satisfy 0 <= cx <= W-1, 0 <= cy <= H-1");
  if (cx > 32767 || cy > 32767)
    return fail(LPF_E_UNSUPPORTED, std::string(fn) + ": cutoff above 32767 (vectors are int16)");
  if (mask < 1 || mask > 3) return fail(LPF_E_INVAL, std::string(fn) + ": phase_mask must be 1, 2 or 3");
  return LPF_OK;
}

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
  if (e == hipSuccess) e = prepare_delta_kernels(kDeltaLdsMax);
  if (e == hipSuccess) e = prepare_step_kernels(kDeltaLdsMax);
  if (e == hipSuccess) e = prepare_s2_kernels(kMaxLds);
  if (e == hipSuccess) e = prepare_lpf3_kernels(kMaxLds);
  if (e != hipSuccess) {
    delete c;
    return hip_fail(e, "lpf_ctx_create: kernel attributes");
  }
  if (hip_device >= kMaxDevices) {
    delete c;
    return fail(LPF_E_UNSUPPORTED, "lpf_ctx_create: device index above 63");
  }
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[hip_device]) {
      void *p = nullptr;
      e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p) {
        delete c;
        return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                        "lpf_ctx_create: address of the no-alloc scratch");
      }
      g_scratch_ptr[hip_device] = (uint32_t *)p;
    }
    c->noalloc_scratch = g_scratch_ptr[hip_device];
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
      (void)hipFree(kv.second.chains);
      (void)hipFree(kv.second.mems);
      (void)hipFree(kv.second.bin_off);
    }
    release_batch_graphs(c);
    for (auto &kv : c->delta_plans) {
      (void)hipFree(kv.second.vecs);
      (void)hipFree(kv.second.chunk_off);
      (void)hipFree(kv.second.runs);
    }
    for (auto &kv : c->diag_plans) {
      (void)hipFree(kv.second.groups);
      (void)hipFree(kv.second.rows);
      (void)hipFree(kv.second.chunk_off);
    }
    for (auto &kv : c->vec3) {
      (void)hipFree(kv.second.vec);
      (void)hipFree(kv.second.woff);
      for (auto &w : kv.second.walk) (void)hipFree(w.second);
    }
    for (auto &kv : c->s2_plans) {
      (void)hipFree(kv.second.fams);
      (void)hipFree(kv.second.groups);
      (void)hipFree(kv.second.vec);
    }
    c->ext.release();
    c->ext3.release();
    c->s2ext.release();
    c->s2acc.release();
    c->sext.release();
    c->rank_buf.release();
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

namespace {
lpf_status full_impl(lpf_ctx c, const uint64_t *bits, int W, int H, int cx, int cy,
                     unsigned phase_mask, int out_layout, uint32_t *counts, void *stream,
                     bool skip, const uint64_t *sample = nullptr) {
  if (!c) return fail(LPF_E_INVAL, "lpf_full: ctx is NULL");
  if (!bits || !counts) return fail(LPF_E_INVAL, "lpf_full: NULL buffer");
  if (W < 1 || H < 1 || W > 65535 || H > 65535) return fail(LPF_E_INVAL, "lpf_full: W/H out of range");
  if (cx < 0 || cy < 0 || cx > W - 1 || cy > H - 1)
    return fail(LPF_E_INVAL, "lpf_full: cutoff must satisfy 0 <= cx <= W-1, 0 <= cy <= H-1");
  if (cx > 32767 || cy > 32767)
    return fail(LPF_E_UNSUPPORTED, "lpf_full: cutoff above 32767 (vectors are int16)");
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
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  const int ext_rows = sh.glob ? sh.lds_rows : H;
  if ((e = c->ext.ensure((size_t)ext_rows * sh.we * sizeof(uint32_t))) != hipSuccess)
    return hip_fail(e, "lpf_full: scratch");
  uint32_t *ext = (uint32_t *)c->ext.p;
  if ((e = launch_ext(bits, W, H, sh.we, ext, s, ext_rows)) != hipSuccess)
    return hip_fail(e, "lpf_full: ext");
  FullImg I = make_img(*plan, ext, counts, W, H, cx, cy, out_layout);
  if (sample) {
    if ((e = c->sext.ensure((size_t)H * sh.we * sizeof(uint32_t))) != hipSuccess)
      return hip_fail(e, "lpf_full_sampled: scratch");
    if ((e = launch_ext(sample, W, H, sh.we, (uint32_t *)c->sext.p, s)) != hipSuccess)
      return hip_fail(e, "lpf_full_sampled: ext");
    I.sample = (const uint32_t *)c->sext.p;
    I.sample_stride = sh.we;
  }
  if ((e = launch_full(I, sh, phase_mask, skip, s)) != hipSuccess) return hip_fail(e, "lpf_full: kernel");
  return LPF_OK;
}
}  // namespace

lpf_status lpf_full(lpf_ctx c, const uint64_t *bits, int W, int H, int cx, int cy,
                    unsigned phase_mask, int out_layout, uint32_t *counts, void *stream) {
  return full_impl(c, bits, W, H, cx, cy, phase_mask, out_layout, counts, stream, false);
}

lpf_status lpf_full_noalloc(lpf_ctx c, const uint64_t *bits, int W, int H, int cx, int cy,
                            unsigned phase_mask, int out_layout, uint32_t *counts, void *stream) {
  if (!c) return fail(LPF_E_INVAL, "lpf_full_noalloc: ctx is NULL");
  if (!bits || !counts) return fail(LPF_E_INVAL, "lpf_full_noalloc: NULL buffer");
  if (W < 1 || H < 1 || W > 65535 || H > 65535)
    return fail(LPF_E_INVAL, "lpf_full_noalloc: W/H out of range");
  if (cx < 0 || cy < 0 || cx > W - 1 || cy > H - 1)
    return fail(LPF_E_INVAL, "lpf_full_noalloc: cutoff must satisfy 0 <= cx <= W-1, 0 <= cy <= H-1");
  if (cx > 32767 || cy > 32767)
    return fail(LPF_E_UNSUPPORTED, "lpf_full_noalloc: cutoff above 32767 (vectors are int16)");
  if (phase_mask < 1 || phase_mask > 3)
    return fail(LPF_E_INVAL, "lpf_full_noalloc: phase_mask must be 1, 2 or 3");
  if (out_layout != LPF_OUT_HALF && out_layout != LPF_OUT_GRID)
    return fail(LPF_E_INVAL, "lpf_full_noalloc: out_layout");
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->dev);
  if (!g.ok) return fail(LPF_E_DEVICE, "lpf_full_noalloc: cannot select the context's device");
  if (!c->noalloc_scratch) return fail(LPF_E_DEVICE, "lpf_full_noalloc: no scratch address");
  FullShape sh{};
  std::string why;
  if (!choose_shape(c, W, H, cx, cy, sh, why))
    return fail(LPF_E_UNSUPPORTED, "lpf_full_noalloc: " + why);
  if (full_lds_bytes(sh, sh.wpg) > (size_t)kMaxLds)
    return fail(LPF_E_UNSUPPORTED, "lpf_full_noalloc: tile shape needs more than 160 KiB of LDS");
  if (sh.glob)
    return fail(LPF_E_UNSUPPORTED,
                "lpf_full_noalloc: halo rows exceed on-chip staging (use lpf_full)");
  if ((size_t)H * sh.we > kNoAllocWords)
    return fail(LPF_E_UNSUPPORTED,
                "lpf_full_noalloc: extended image of " + std::to_string((size_t)H * sh.we * 4) +
                    " bytes exceeds the fixed scratch of " + std::to_string(kNoAllocWords * 4) +
                    " bytes (H * (words per row + cx/32 + 1) * 4)");
  const int64_t nv = (int64_t)(cx + 1) * (cy + 1) + (int64_t)cx * cy;
  // bins (one workgroup each): two per CU, at most kSlotWords / 2 vectors each
  int cus = 256;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->dev);
  int64_t nb = std::min<int64_t>(nv, 2 * (int64_t)cus);
  nb = std::max<int64_t>(nb, (2 * nv + kSlotWords - 1) / kSlotWords);
  if (nv > (int64_t)1 << 30 || nb > (int64_t)1 << 24)
    return fail(LPF_E_UNSUPPORTED, "lpf_full_noalloc: too many vectors");
  sh.nbins = (int)nb;
  hipStream_t s = (hipStream_t)stream;
  uint32_t *ext = c->noalloc_scratch;
  hipError_t e;
  if ((e = launch_ext(bits, W, H, sh.we, ext, s)) != hipSuccess)
    return hip_fail(e, "lpf_full_noalloc: ext");
  FullImg I{};
  I.E = ext;
  I.out = counts;
  I.W = W;
  I.H = H;
  I.cx = cx;
  I.cy = cy;
  I.R = sh.R;
  I.S = sh.S;
  I.we = sh.we;
  I.rst = sh.rst;
  I.tile = sh.tile;
  I.ntiles = sh.ntiles;
  I.lds_rows = sh.lds_rows;
  I.nv = (int)nv;
  I.layout = out_layout;
  I.nbins = sh.nbins;
  I.nwb = sh.nwb;
  if ((e = launch_full_canon(I, sh, phase_mask, s)) != hipSuccess)
    return hip_fail(e, "lpf_full_noalloc: kernel");
  return LPF_OK;
}

lpf_status lpf_peak_probe(lpf_ctx c, int kind, int64_t iters, int nwg, uint32_t *sink,
                          double *work, void *stream) {
  if (!c) return fail(LPF_E_INVAL, "lpf_peak_probe: ctx is NULL");
  if (kind < 0 || kind > 4) return fail(LPF_E_INVAL, "lpf_peak_probe: kind must be 0..4");
  if (iters < 1 || iters > ((int64_t)1 << 40)) return fail(LPF_E_INVAL, "lpf_peak_probe: iters");
  if (nwg < 1 || nwg > 65536) return fail(LPF_E_INVAL, "lpf_peak_probe: nwg must be 1..65536");
  if (!sink) return fail(LPF_E_INVAL, "lpf_peak_probe: sink is NULL");
  DeviceGuard g(c->dev);
  if (!g.ok) return fail(LPF_E_DEVICE, "lpf_peak_probe: cannot select the context's device");
  hipError_t e = launch_probe(kind, iters, nwg, sink, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "lpf_peak_probe");
  if (work) *work = probe_work(kind, iters, nwg);
  return LPF_OK;
}

lpf_status lpf_full_enhanced(lpf_ctx c, const uint64_t *bits, int W, int H, int cx, int cy,
                             unsigned phase_mask, int out_layout, uint32_t *counts,
                             void *stream) {
  return full_impl(c, bits, W, H, cx, cy, phase_mask, out_layout, counts, stream, true);
}

lpf_status lpf_full_sampled(lpf_ctx c, const uint64_t *bits, int W, int H, int cx, int cy,
                            unsigned phase_mask, int out_layout, const uint64_t *sample,
                            uint32_t *counts, void *stream) {
  if (!sample) return fail(LPF_E_INVAL, "lpf_full_sampled: sample is NULL");
  return full_impl(c, bits, W, H, cx, cy, phase_mask, out_layout, counts, stream, false, sample);
}

// Tile-shape override used by the autotuner and by tests (0 = automatic choice).
lpf_status lpf_set_full_shape(lpf_ctx c, int R, int S, int waves_per_group, int lds_bytes) {
  if (!c) return fail(LPF_E_INVAL, "lpf_set_full_shape: ctx is NULL");
  auto pow2ok = [](int v, int hi) { return v == 0 || (v >= 1 && v <= hi && (v & (v - 1)) == 0); };
  if (!pow2ok(R, 16) || !pow2ok(S, 64) || waves_per_group < 0 || waves_per_group > 16 ||
      lds_bytes < 0 || lds_bytes > kMaxLds)
    return fail(LPF_E_INVAL, "lpf_set_full_shape: R in {1..16}, S in {1..64} powers of two, "
                             "waves 1..16, lds <= 160 KiB (0 = automatic)");
  std::lock_guard<std::mutex> lk(c->mu);
  c->force_R = R;
  c->force_S = S;
  c->force_wpg = waves_per_group;
  c->force_lds = lds_bytes;
  return LPF_OK;
}

lpf_status lpf_delta_swap(lpf_ctx c, const uint64_t *bits, int W, int H, int cx, int cy,
                          unsigned phase_mask, const int32_t *swaps, int n, int32_t *delta,
                          void *stream) {
  if (!c) return fail(LPF_E_INVAL, "lpf_delta_swap: ctx is NULL");
  lpf_status st = check_image_args("lpf_delta_swap", W, H, cx, cy, phase_mask);
  if (st != LPF_OK) return st;
  if (n < 0 || n > (1 << 24)) return fail(LPF_E_INVAL, "lpf_delta_swap: n outside [0, 2^24]");
  if (n == 0) return LPF_OK;
  if (!bits || !swaps || !delta) return fail(LPF_E_INVAL, "lpf_delta_swap: NULL buffer");
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->dev);
  if (!g.ok) return fail(LPF_E_DEVICE, "lpf_delta_swap: cannot select the context's device");
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  // offset rows where their table fits (cutoffs up to 255), else the run-based kernel
  DiagPlan *dp = nullptr;
  if (!c->force_run_delta) {
    if ((st = get_diag_plan(c, cx, cy, delta_chunks(n), dp)) != LPF_OK) return st;
  }
  if (dp && dp->ok) {
    const DiagGeo geo = diag_geometry(W, H, cx, cy);
    if ((e = c->ext3.ensure((size_t)geo.total * 4)) != hipSuccess)
      return hip_fail(e, "lpf_delta_swap: scratch");
    if ((e = launch_dframe(bits, W, H, geo, (uint32_t *)c->ext3.p, s)) != hipSuccess)
      return hip_fail(e, "lpf_delta_swap: frames");
    DiagLaunch L{};
    L.F = (const uint32_t *)c->ext3.p;
    L.geo = geo;
    L.bits = bits;
    L.W = W;
    L.H = H;
    L.cand = reinterpret_cast<const int2 *>(swaps);
    L.K = n;
    L.groups = dp->groups;
    L.chunk_off = dp->chunk_off;
    L.rows = dp->rows;
    L.nchunks = dp->nchunks;
    L.phase_mask = phase_mask;
    L.nv = (int)lpf_num_vectors(cx, cy);
    L.delta_out = delta;
    L.use_lds = (int64_t)geo.total * 4 <= kDeltaLdsMax;
    if ((e = launch_delta_diag(L, s)) != hipSuccess) return hip_fail(e, "lpf_delta_swap: kernel");
    return LPF_OK;
  }
  DeltaPlan *plan = nullptr;
  if ((st = get_delta_plan(c, W, H, cx, cy, delta_chunks(n), plan)) != LPF_OK) return st;
  if ((e = c->ext3.ensure((size_t)plan->geo.total * 4)) != hipSuccess)
    return hip_fail(e, "lpf_delta_swap: scratch");
  if ((e = launch_ext3(bits, W, H, plan->geo, (uint32_t *)c->ext3.p, s)) != hipSuccess)
    return hip_fail(e, "lpf_delta_swap: ext3");
  DeltaLaunch L{};
  L.E = (const uint32_t *)c->ext3.p;
  L.geo = plan->geo;
  L.bits = bits;
  L.W = W;
  L.H = H;
  L.cand = reinterpret_cast<const int2 *>(swaps);
  L.K = n;
  L.vecs = plan->vecs;
  L.chunk_off = plan->chunk_off;
  L.runs = plan->runs;
  L.phase_mask = phase_mask;
  L.nv = (int)plan->nv;
  L.delta_out = delta;
  L.nchunks = plan->nchunks;
  L.use_lds = plan->use_lds;
  if ((e = launch_delta(L, s)) != hipSuccess) return hip_fail(e, "lpf_delta_swap: kernel");
  return LPF_OK;
}

lpf_status lpf_set_delta_method(lpf_ctx c, int method) {
  if (!c) return fail(LPF_E_INVAL, "lpf_set_delta_method: ctx is NULL");
  if (method != LPF_SWAP_AUTO && method != LPF_SWAP_RUNS)
    return fail(LPF_E_INVAL, "lpf_set_delta_method: method must be LPF_SWAP_AUTO or LPF_SWAP_RUNS");
  std::lock_guard<std::mutex> lk(c->mu);
  c->force_run_delta = method == LPF_SWAP_RUNS;
  return LPF_OK;
}

int64_t lpf_num_vectors3(int cx, int cy, int cz) {
  if (cx < 0 || cy < 0 || cz < 0) return -1;
  return lpf_num_vectors(cx, cy) + (int64_t)cz * (2 * cx + 1) * (2 * cy + 1);
}

lpf_status lpf_vectors3(int cx, int cy, int cz, int16_t *dxdydz) {
  if (cx < 0 || cy < 0 || cz < 0 || cx > 32767 || cy > 32767 || cz > 32767)
    return fail(LPF_E_INVAL, "lpf_vectors3: cutoff");
  if (!dxdydz) return fail(LPF_E_INVAL, "lpf_vectors3: NULL buffer");
  std::vector<int16_t> can;
  canonical_vectors(cx, cy, can);
  size_t i = 0;
  for (size_t j = 0; j < can.size(); j += 2, ++i) {
    dxdydz[3 * i] = can[j];
    dxdydz[3 * i + 1] = can[j + 1];
    dxdydz[3 * i + 2] = 0;
  }
  for (int dz = 1; dz <= cz; ++dz)
    for (int dy = -cy; dy <= cy; ++dy)
      for (int dx = -cx; dx <= cx; ++dx, ++i) {
        dxdydz[3 * i] = (int16_t)dx;
        dxdydz[3 * i + 1] = (int16_t)dy;
        dxdydz[3 * i + 2] = (int16_t)dz;
      }
  return LPF_OK;
}

lpf_status lpf_full3d(lpf_ctx c, const uint64_t *bits, int W, int H, int D, int cx, int cy,
                      int cz, unsigned phase_mask, uint32_t *counts, void *stream) {
  if (!c) return fail(LPF_E_INVAL, "lpf_full3d: ctx is NULL");
  if (!bits || !counts) return fail(LPF_E_INVAL, "lpf_full3d: NULL buffer");
  if (W < 1 || H < 1 || D < 1 || W > 65535 || H > 65535 || D > 65535 || (int64_t)H * D > 65535LL * 65535LL)
    return fail(LPF_E_INVAL, "lpf_full3d: W/H/D out of range");
  if (cx < 0 || cy < 0 || cz < 0 || cx > W - 1 || cy > H - 1 || cz > D - 1 || cx > 32767 ||
      cy > 32767 || cz > 32767)
    return fail(LPF_E_INVAL, "lpf_full3d: cutoff must satisfy 0 <= c <= size - 1 on each axis");
  if (phase_mask < 1 || phase_mask > 3) return fail(LPF_E_INVAL, "lpf_full3d: phase_mask must be 1, 2 or 3");
  const int64_t nv = lpf_num_vectors3(cx, cy, cz);
  if (nv > (int64_t)1 << 30) return fail(LPF_E_UNSUPPORTED, "lpf_full3d: too many vectors");
  if ((int64_t)W * H * D > ((int64_t)1 << 32) - 1)
    return fail(LPF_E_UNSUPPORTED, "lpf_full3d: more than 2^32 - 1 voxels (uint32 counts)");
  const int swd = (W + 31) / 32;
  const int R = std::min(16, next_pow2(swd));
  const int S = next_pow2((swd + R - 1) / R);
  if (S > 64) return fail(LPF_E_UNSUPPORTED, "lpf_full3d: rows too wide (W > 32768)");
  const int we = S * R + (cx >> 5) + 1;
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->dev);
  if (!g.ok) return fail(LPF_E_DEVICE, "lpf_full3d: cannot select the context's device");
  hipError_t e;
  lpf_ctx_s::Vec3 *v3p = nullptr;
  auto key = std::make_tuple(cx, cy, cz);
  auto it = c->vec3.find(key);
  if (it != c->vec3.end()) {
    v3p = &it->second;
  } else {
    // launch order: longest segments first, so that the waves of a workgroup walk segments of
    // equal length and the long ones start early; each vector's voxel-table entries: n + 1
    // rounded up to even
    std::vector<int16_t> v3((size_t)nv * 3);
    lpf_vectors3(cx, cy, cz, v3.data());
    std::vector<int4> hv(nv);
    for (int64_t i = 0; i < nv; ++i) hv[i] = make_int4(v3[3 * i], v3[3 * i + 1], v3[3 * i + 2], (int)i);
    auto len = [](const int4 &a) { return std::max(std::abs(a.x), std::max(std::abs(a.y), std::abs(a.z))); };
    std::stable_sort(hv.begin(), hv.end(), [&](const int4 &a, const int4 &b) { return len(a) > len(b); });
    std::vector<int> woff(nv);
    lpf_ctx_s::Vec3 rec;
    for (int64_t i = 0; i < nv; ++i) {
      woff[i] = (int)rec.nwalk;
      rec.nwalk += (len(hv[i]) + 2) & ~1;
    }
    if (rec.nwalk > ((int64_t)1 << 30)) return fail(LPF_E_UNSUPPORTED, "lpf_full3d: voxel table too large");
    if ((e = hipMalloc(&rec.vec, sizeof(int4) * nv)) != hipSuccess) return hip_fail(e, "lpf_full3d: vectors");
    if ((e = hipMalloc(&rec.woff, sizeof(int) * nv)) != hipSuccess ||
        (e = hipMemcpy(rec.vec, hv.data(), sizeof(int4) * nv, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(rec.woff, woff.data(), sizeof(int) * nv, hipMemcpyHostToDevice)) != hipSuccess) {
      (void)hipFree(rec.vec);
      (void)hipFree(rec.woff);
      return hip_fail(e, "lpf_full3d: vectors");
    }
    v3p = &(c->vec3[key] = rec);
  }
  const int4 *vec = v3p->vec;
  hipStream_t s = (hipStream_t)stream;
  const int rows = H * D;
  if ((e = c->ext.ensure((size_t)rows * we * sizeof(uint32_t))) != hipSuccess)
    return hip_fail(e, "lpf_full3d: scratch");
  if ((e = launch_ext(bits, W, rows, we, (uint32_t *)c->ext.p, s)) != hipSuccess)
    return hip_fail(e, "lpf_full3d: ext");
  // slabs in LDS when at least cz + 1 planes fit half the LDS (two workgroups per CU) or all
  // of it; otherwise rows from global memory
  // rows rst (odd) dwords apart, so that a wave's consecutive start rows fall in distinct banks;
  // planes ps dwords apart, with a gap that makes the jump over the 2 cy halo rows between two
  // planes a multiple of 32 dwords (the banks one half-wave's reads spread over), so that rows
  // on both sides of a plane boundary do too
  const int rst = we | 1;
  const int64_t ps64 = (int64_t)(H + 2 * cy) * rst + ((32 - (2LL * cy * rst) % 32) % 32);
  const size_t plane = (size_t)ps64 * sizeof(uint32_t);
  size_t budget = kMaxLds / 2;
  if ((size_t)(cz + 1) * plane > budget) budget = kMaxLds;
  if ((size_t)(cz + 1) * plane <= budget) {
    const int zb = (int)std::min<int64_t>(D, (int64_t)(budget / plane) - cz);
    // the voxel table of this geometry: built by the first call that needs it (enqueued before
    // that call's kernel), never written again
    const int ps = (int)ps64;
    int2 *&walk = v3p->walk[std::make_pair(ps, rst)];
    const bool build = walk == nullptr;
    if (build && (e = hipMalloc(&walk, (size_t)v3p->nwalk * sizeof(int2))) != hipSuccess) {
      walk = nullptr;
      v3p->walk.erase(std::make_pair(ps, rst));
      return hip_fail(e, "lpf_full3d: voxel table");
    }
    // two start rows per lane for short segments (measured at 100^3: cutoff 16, about 14 voxels
    // per segment, 0.98 ms against 1.02 with one; the full in-plane domain of the cuts, about 67,
    // 4.74 ms with one against 4.96 with two)
    const int rpl = v3p->nwalk < 32 * nv ? 2 : 1;
    e = launch_lpf3_slab((const uint32_t *)c->ext.p, W, H, D, we, R, S, rst, ps, zb, cz, cy, vec,
                         v3p->woff, walk, build, rpl, (int)nv, phase_mask, counts, s);
    if (e != hipSuccess && build) {  // the table may not have been written: drop it
      (void)hipFree(walk);
      v3p->walk.erase(std::make_pair(ps, rst));
    }
  } else {
    e = launch_lpf3((const uint32_t *)c->ext.p, W, H, D, we, R, S, vec, (int)nv, phase_mask,
                    counts, s);
  }
  if (e != hipSuccess) return hip_fail(e, "lpf_full3d: kernel");
  return LPF_OK;
}

lpf_status lpf_s2(lpf_ctx c, const uint64_t *bits, int W, int H, int cx, int cy,
                  unsigned phase_mask, int out_layout, uint32_t *counts, void *stream) {
  if (!c) return fail(LPF_E_INVAL, "lpf_s2: ctx is NULL");
  lpf_status st = check_image_args("lpf_s2", W, H, cx, cy, phase_mask);
  if (st != LPF_OK) return st;
  if (!bits || !counts) return fail(LPF_E_INVAL, "lpf_s2: NULL buffer");
  if (out_layout != LPF_OUT_HALF && out_layout != LPF_OUT_GRID)
    return fail(LPF_E_INVAL, "lpf_s2: out_layout");
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->dev);
  if (!g.ok) return fail(LPF_E_DEVICE, "lpf_s2: cannot select the context's device");
  S2Plan *plan = nullptr;
  if ((st = get_s2_plan(c, W, H, cx, cy, plan)) != LPF_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  // two accumulators of ncap entries, zero on (re)allocation; each call clears the one it does
  // not use for the next
  if ((e = ensure_zeroed(c->s2acc, 2 * (size_t)plan->nv * sizeof(uint32_t), s)) != hipSuccess)
    return hip_fail(e, "lpf_s2: scratch");
  const int64_t ncap = (int64_t)(c->s2acc.bytes / (2 * sizeof(uint32_t)));
  S2Launch L{};
  L.E = reinterpret_cast<const uint32_t *>(bits);  // the kernel extends the rows as it stages them
  L.W = W;
  L.H = H;
  L.we = plan->we;
  L.swd = plan->swd;
  L.swdp = plan->swdp;
  L.J = plan->J;
  L.rb = plan->rb;
  L.nrb = plan->nrb;
  L.rstB = plan->rstB;
  L.ngroups = plan->ngroups;
  L.cx = cx;
  L.cy = cy;
  L.layout = out_layout;
  L.fams = plan->fams;
  L.groups = plan->groups;
  L.lds_bytes = plan->lds;
  L.acc = (uint32_t *)c->s2acc.p + (size_t)c->s2half * ncap;
  L.clear = (uint32_t *)c->s2acc.p + (size_t)(c->s2half ^ 1) * ncap;
  L.ncap = ncap;
  L.nv = plan->nv;
  L.phase_mask = phase_mask;
  L.out = counts;
  if ((e = launch_s2_full(L, s)) != hipSuccess) return hip_fail(e, "lpf_s2: kernel");
  c->s2half ^= 1;
  return LPF_OK;
}

lpf_status lpf_s2_delta_swap(lpf_ctx c, const uint64_t *bits, int W, int H, int cx, int cy,
                             unsigned phase_mask, const int32_t *swaps, int n, int32_t *delta,
                             void *stream) {
  if (!c) return fail(LPF_E_INVAL, "lpf_s2_delta_swap: ctx is NULL");
  lpf_status st = check_image_args("lpf_s2_delta_swap", W, H, cx, cy, phase_mask);
  if (st != LPF_OK) return st;
  if (n < 0 || n > (1 << 24)) return fail(LPF_E_INVAL, "lpf_s2_delta_swap: n outside [0, 2^24]");
  if (n == 0) return LPF_OK;
  if (!bits || !swaps || !delta) return fail(LPF_E_INVAL, "lpf_s2_delta_swap: NULL buffer");
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->dev);
  if (!g.ok) return fail(LPF_E_DEVICE, "lpf_s2_delta_swap: cannot select the context's device");
  S2Plan *plan = nullptr;
  if ((st = get_s2_plan(c, W, H, cx, cy, plan)) != LPF_OK) return st;
  hipError_t e = launch_s2_delta(bits, W, H, reinterpret_cast<const int2 *>(swaps), n, plan->vec,
                                 plan->nv, phase_mask, delta, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "lpf_s2_delta_swap: kernel");
  return LPF_OK;
}

namespace {
lpf_status anneal_create(lpf_ctx c, uint64_t *bits, int W, int H, int cx, int cy,
                         unsigned phase_mask, uint32_t *counts, const uint32_t *target, int64_t Nt,
                         uint64_t seed, uint64_t step0, const int32_t *pos, int n1, double *e_dev,
                         lpf_anneal *out, void *stream, bool s2,
                         const uint64_t *sample = nullptr) {
  if (!out) return fail(LPF_E_INVAL, "lpf_anneal_create: out is NULL");
  *out = nullptr;
  if (!c) return fail(LPF_E_INVAL, "lpf_anneal_create: ctx is NULL");
  lpf_status st = check_image_args("lpf_anneal_create", W, H, cx, cy, phase_mask);
  if (st != LPF_OK) return st;
  if (!bits || !counts || !target || !e_dev) return fail(LPF_E_INVAL, "lpf_anneal_create: NULL buffer");
  if (Nt < 1 || Nt > ((int64_t)1 << 40)) return fail(LPF_E_INVAL, "lpf_anneal_create: Nt");
  const int64_t N = (int64_t)W * H;
  if (N < 2 || N > ((int64_t)1 << 26)) return fail(LPF_E_INVAL, "lpf_anneal_create: W*H outside [2, 2^26]");
  if (pos && (n1 < 1 || n1 > N - 1)) return fail(LPF_E_INVAL, "lpf_anneal_create: n1");
  if (std::max(cx, cy) > 16383)
    return fail(LPF_E_INVAL, "lpf_anneal_create: cutoff above 16383 (per-candidate deltas are int16)");
  {
    // exact energy sums: |dL| <= 2 (n + 1) per term, so every partial sum of
    // dL (Nt (dL + 2L) - 2 N T) is below nterms * dmax * Nt * (dmax + 4N); keep it in int64
    const __int128 dmax = s2 ? 6 : 2 * ((__int128)std::max(cx, cy) + 1);
    const __int128 bound = (__int128)nph_of(phase_mask) * lpf_num_vectors(cx, cy) * dmax *
                           (__int128)Nt * (dmax + 4 * (__int128)W * H);
    if (bound > (__int128)INT64_MAX)
      return fail(LPF_E_UNSUPPORTED, "lpf_anneal_create: cell, cutoff and Nt too large for exact int64 energy sums");
  }
  int64_t Neff = N;
  if (sample) {
    if (std::max(cx, cy) > 126)
      return fail(LPF_E_UNSUPPORTED, "lpf_anneal_create_sampled: cutoff above 126 (the position set rides on the placement counts)");
    // the number of sampled positions (bits past W ignored)
    const int wpr = (W + 63) / 64;
    std::vector<uint64_t> hm((size_t)wpr * H);
    DeviceGuard g0(c->dev);
    hipError_t e0 = hipMemcpyAsync(hm.data(), sample, hm.size() * 8, hipMemcpyDeviceToHost,
                                   (hipStream_t)stream);
    if (e0 == hipSuccess) e0 = hipStreamSynchronize((hipStream_t)stream);
    if (e0 != hipSuccess) return hip_fail(e0, "lpf_anneal_create_sampled: position set");
    Neff = 0;
    for (int y = 0; y < H; ++y)
      for (int w = 0; w < wpr; ++w) {
        uint64_t v = hm[(size_t)y * wpr + w];
        const int valid = std::min(64, W - 64 * w);
        if (valid < 64) v &= (1ull << valid) - 1ull;
        Neff += __builtin_popcountll(v);
      }
    if (Neff < 1) return fail(LPF_E_INVAL, "lpf_anneal_create_sampled: empty position set");
  }
  // full evaluation for the initial counts (also validates the tile shape)
  st = s2       ? lpf_s2(c, bits, W, H, cx, cy, phase_mask, LPF_OUT_HALF, counts, stream)
       : sample ? lpf_full_sampled(c, bits, W, H, cx, cy, phase_mask, LPF_OUT_HALF, sample,
                                   counts, stream)
                : lpf_full(c, bits, W, H, cx, cy, phase_mask, LPF_OUT_HALF, counts, stream);
  if (st != LPF_OK) return st;
  lpf_anneal a = new (std::nothrow) lpf_anneal_s();
  if (!a) return fail(LPF_E_NOMEM, "lpf_anneal_create: host memory");
  a->ctx = c;
  a->s2 = s2;
  a->sample = sample;
  a->Neff = Neff;
  a->W = W; a->H = H; a->cx = cx; a->cy = cy; a->mask = phase_mask;
  a->bits = bits; a->counts = counts; a->target = target; a->e = e_dev;
  a->Nt = Nt; a->seed = seed;
  if (sample) {
    std::string why;
    if (!records_fit(a, nullptr, &why)) {
      delete a;
      return fail(LPF_E_UNSUPPORTED, "lpf_anneal_create_sampled: " + why);
    }
  }
  DeviceGuard g(c->dev);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  AnnealDev host{};
  host.step = step0;
  host.last_a = -1;
  host.last_b = -1;
  a->host_step = step0;
  if ((e = hipMalloc(&a->dev, sizeof(AnnealDev))) != hipSuccess ||
      (e = hipMalloc(&a->pos, sizeof(int32_t) * (size_t)N)) != hipSuccess) {
    lpf_anneal_destroy(a);
    return hip_fail(e, "lpf_anneal_create: allocation");
  }
  host.pos1 = a->pos;
  host.pos0 = a->pos;  // set below once n1 is known
  if (pos) {
    host.n1 = n1;
    host.n0 = (int32_t)(N - n1);
    host.pos0 = a->pos + n1;
    if ((e = hipMemcpyAsync(a->pos, pos, sizeof(int32_t) * (size_t)N, hipMemcpyDeviceToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(a->dev, &host, sizeof(AnnealDev), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess) {
      lpf_anneal_destroy(a);
      return hip_fail(e, "lpf_anneal_create: state upload");
    }
  } else {
    // lists in ascending order: count ones first, then place phase-0 list after the ones
    int32_t *tmp1 = nullptr;
    if ((e = hipMalloc(&tmp1, sizeof(int32_t) * (size_t)N)) != hipSuccess) {
      lpf_anneal_destroy(a);
      return hip_fail(e, "lpf_anneal_create: allocation");
    }
    AnnealDev scratch = host;
    scratch.pos1 = a->pos;
    scratch.pos0 = tmp1;
    int32_t n1h = 0;
    if ((e = hipMemcpyAsync(a->dev, &scratch, sizeof(AnnealDev), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = launch_init_lists(a->dev, bits, W, H, s)) != hipSuccess ||
        (e = hipMemcpyAsync(&n1h, &a->dev->n1, sizeof(int32_t), hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess) {
      (void)hipFree(tmp1);
      lpf_anneal_destroy(a);
      return hip_fail(e, "lpf_anneal_create: pixel lists");
    }
    if (n1h < 1 || n1h > N - 1) {
      (void)hipFree(tmp1);
      lpf_anneal_destroy(a);
      return fail(LPF_E_INVAL, "lpf_anneal_create: the image must contain both phases");
    }
    host.n1 = n1h;
    host.n0 = (int32_t)(N - n1h);
    host.pos0 = a->pos + n1h;
    if ((e = hipMemcpyAsync(a->pos + n1h, tmp1, sizeof(int32_t) * (size_t)(N - n1h), hipMemcpyDeviceToDevice, s)) != hipSuccess ||
        (e = hipMemcpyAsync(a->dev, &host, sizeof(AnnealDev), hipMemcpyHostToDevice, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess) {
      (void)hipFree(tmp1);
      lpf_anneal_destroy(a);
      return hip_fail(e, "lpf_anneal_create: pixel lists");
    }
    (void)hipFree(tmp1);
  }
  const int nph = nph_of(phase_mask);
  const int64_t nv = lpf_num_vectors(cx, cy);
  if ((e = launch_lse(counts, target, nph * nv, Neff, Nt, e_dev, s)) != hipSuccess) {
    lpf_anneal_destroy(a);
    return hip_fail(e, "lpf_anneal_create: energy");
  }
  *out = a;
  return LPF_OK;
}
}  // namespace

lpf_status lpf_anneal_create(lpf_ctx c, uint64_t *bits, int W, int H, int cx, int cy,
                             unsigned phase_mask, uint32_t *counts, const uint32_t *target,
                             int64_t Nt, uint64_t seed, uint64_t step0, const int32_t *pos,
                             int n1, double *e_dev, lpf_anneal *out, void *stream) {
  return anneal_create(c, bits, W, H, cx, cy, phase_mask, counts, target, Nt, seed, step0, pos,
                       n1, e_dev, out, stream, false);
}

lpf_status lpf_anneal_create_s2(lpf_ctx c, uint64_t *bits, int W, int H, int cx, int cy,
                                unsigned phase_mask, uint32_t *counts, const uint32_t *target,
                                int64_t Nt, uint64_t seed, uint64_t step0, const int32_t *pos,
                                int n1, double *e_dev, lpf_anneal *out, void *stream) {
  return anneal_create(c, bits, W, H, cx, cy, phase_mask, counts, target, Nt, seed, step0, pos,
                       n1, e_dev, out, stream, true);
}

lpf_status lpf_anneal_create_sampled(lpf_ctx c, uint64_t *bits, int W, int H, int cx, int cy,
                                     unsigned phase_mask, const uint64_t *sample,
                                     uint32_t *counts, const uint32_t *target, int64_t Nt,
                                     uint64_t seed, uint64_t step0, const int32_t *pos, int n1,
                                     double *e_dev, lpf_anneal *out, void *stream) {
  if (!sample) {
    if (out) *out = nullptr;
    return fail(LPF_E_INVAL, "lpf_anneal_create_sampled: sample is NULL");
  }
  return anneal_create(c, bits, W, H, cx, cy, phase_mask, counts, target, Nt, seed, step0, pos,
                       n1, e_dev, out, stream, false, sample);
}

namespace {

lpf_status step_args(const char *fn, lpf_anneal a, int K, int proposal) {
  if (!a) return fail(LPF_E_INVAL, std::string(fn) + ": state is NULL");
  if (K < 1 || K > (1 << 20)) return fail(LPF_E_INVAL, std::string(fn) + ": n_candidates outside [1, 2^20]");
  if (proposal != LPF_PROP_UNIFORM && proposal != LPF_PROP_INTERFACIAL &&
      proposal != LPF_PROP_LEARNED)
    return fail(LPF_E_INVAL, std::string(fn) + ": proposal");
  if (proposal == LPF_PROP_LEARNED && !a->net && !a->scores_ext)
    return fail(LPF_E_INVAL, std::string(fn) + ": learned proposal without lpf_anneal_set_proposal");
  return LPF_OK;
}

// Plans, scratch and the evaluation state of a step with K candidates (records or frames are
// rebuilt on the stream when stale); fills L except the per-step fields.
lpf_status step_setup(lpf_anneal a, int K, int proposal, hipStream_t s, StepLaunch &L,
                      DeltaPlan *&plan, bool &rec) {
  lpf_ctx c = a->ctx;
  hipError_t e;
  rec = !a->s2 && use_records(a);
  L = StepLaunch{};
  L.s2 = a->s2;
  L.records = rec;
  L.rounds = step_rounds(K, true);
  plan = nullptr;
  lpf_status st;
  if (a->s2) {
    S2Plan *sp = nullptr;
    if ((st = get_s2_plan(c, a->W, a->H, a->cx, a->cy, sp)) != LPF_OK) return st;
    L.s2vec = sp->vec;
    L.use_lds = s2_img_lds(a->W, a->H);
    s2_rounds(L.rounds, sp->nv);
  } else if (rec) {
    if ((st = setup_records(a, s)) != LPF_OK) return st;
    records_rounds(L.rounds);
  } else {
    if ((st = recount_rounds(a, L.rounds, plan)) != LPF_OK) return st;
    if ((st = prepare_eval(a, false, plan->geo, s)) != LPF_OK) return st;
  }
  const int nph = nph_of(a->mask);
  const int64_t nv = lpf_num_vectors(a->cx, a->cy);
  const size_t nterms = (size_t)nph * nv;
  if ((e = a->cand.ensure(sizeof(int2) * 2 * (size_t)K)) != hipSuccess ||
      (e = a->U.ensure(sizeof(double) * 2 * (size_t)K)) != hipSuccess ||
      (e = a->slot.ensure(sizeof(int2) * 2 * (size_t)K)) != hipSuccess ||
      (e = a->S_acc.ensure(sizeof(int64_t) * (size_t)K)) != hipSuccess ||
      (e = a->dl.ensure(sizeof(int16_t) * nterms * (size_t)K)) != hipSuccess ||
      (e = a->ctl.ensure(sizeof(StepCtl))) != hipSuccess ||
      (e = a->ksel.ensure(sizeof(int32_t))) != hipSuccess ||
      (e = a->Tcur.ensure(sizeof(double))) != hipSuccess ||
      (e = a->order.ensure(sizeof(int32_t) * (size_t)K)) != hipSuccess ||
      (e = a->rank_buf.ensure(kRankScratch)) != hipSuccess ||
      (e = ensure_zeroed(a->S0, sizeof(int64_t) * 64, s)) != hipSuccess ||
      (e = ensure_zeroed(a->pre, sizeof(int4) * 128, s)) != hipSuccess)
    return hip_fail(e, "anneal: scratch");
  if (proposal == LPF_PROP_LEARNED) {  // the draw's buffers, so that it allocates nothing
    const int64_t N = (int64_t)a->W * a->H;
    if ((a->net && (e = a->scores.ensure(sizeof(float) * (size_t)N)) != hipSuccess) ||
        (a->beta > 0.0 && ((e = a->cw1.ensure(sizeof(double) * (size_t)N)) != hipSuccess ||
                           (e = a->cw0.ensure(sizeof(double) * (size_t)N)) != hipSuccess ||
                           (e = a->cwb.ensure(sizeof(double) * 4 * (size_t)((N + 1023) / 1024))) != hipSuccess)))
      return hip_fail(e, "anneal: proposal scratch");
  }
  if (plan) {
    L.E = (const uint32_t *)a->E3.p;
    L.geo = plan->geo;
    L.runs = plan->runs;
    L.use_lds = plan->use_lds;
  }
  L.rg = a->rg;
  L.bits = a->bits;
  L.bits_rw = a->bits;
  L.W = a->W;
  L.H = a->H;
  L.cand = (const int2 *)a->cand.p;
  L.slot = (const int2 *)a->slot.p;
  L.U = (const double *)a->U.p;
  L.K = K;
  L.phase_mask = a->mask;
  L.nv = (int)nv;
  L.nterms = (int)nterms;
  L.counts = a->counts;
  L.counts_rw = a->counts;
  L.target = a->target;
  L.N = a->Neff;
  L.Nt = a->Nt;
  L.T = (const double *)a->Tcur.p;
  L.S_acc = (int64_t *)a->S_acc.p;
  L.dl = (int16_t *)a->dl.p;
  L.dl_t = rec ? 1 : K;
  L.dl_k = rec ? (int64_t)nterms : 1;
  L.ctl = (StepCtl *)a->ctl.p;
  L.st = a->dev;
  L.e = a->e;
  L.k_sel = (int32_t *)a->ksel.p;
  L.reset_done = true;  // the draw zeroes the step's sums and control block
  L.ordered = true;     // draws take a from the phase-1 list and b from the phase-0 list
  return LPF_OK;
}

// One step on the stream after step_setup: draw (T from T_sched[step - T_base], or T), ranking,
// rounds, decision, state upkeep.  No allocation and no host synchronisation (capturable, except
// learned proposals, whose re-scoring cadence is kept on the host).
lpf_status step_enqueue(lpf_anneal a, int K, int proposal, StepLaunch &L, DeltaPlan *plan,
                        bool rec, const double *T_sched, int64_t T_base, double T,
                        lpf_step_result *out, int64_t out_base, hipStream_t s,
                        bool allow_next = false) {
  hipError_t e;
  lpf_status st;
  const bool rank = proposal == LPF_PROP_LEARNED && a->rank;
  // the step's half of the double-buffered candidates (the end of a ranked step draws the next
  // step into the other half while it still reads this one)
  const size_t half = (size_t)(a->host_step & 1) * (size_t)K;
  L.cand = (const int2 *)a->cand.p + half;
  L.slot = (const int2 *)a->slot.p + half;
  L.U = (const double *)a->U.p + half;
  // records method, unranked: the draws and round 0 share one launch; ranked: round 0 merges the
  // ranking and does the step's resets
  L.fuse_draw = rec && !rank && L.rounds.size() >= 2 && L.rounds[0].C == 64;
  L.fuse_rank = rec && rank && L.rounds.size() >= 2 && L.rounds[0].C == 64;
  L.S0 = (int64_t *)a->S0.p;
  const bool drawn = L.fuse_rank && a->predrawn;  // made by the previous step's end
  ProposeArgs none{}, args{};
  if ((st = draw_candidates(a, K, proposal, s, (int64_t *)a->S_acc.p, (StepCtl *)a->ctl.p,
                            T_sched, T_base, T, (double *)a->Tcur.p, rank,
                            L.fuse_draw ? &L.draw : drawn ? &none : nullptr, &args)) != LPF_OK)
    return st;
  L.order = nullptr;
  L.draw_next = false;
  if (rank) {
    const uint64_t *keys = (const uint64_t *)a->rank_buf.p;
    int32_t *ord = (int32_t *)a->order.p;
    // records method: round 0 merges the ranking itself and writes the order for later rounds
    L.rank_keys = keys;
    L.order_rw = ord;
    L.T_cur = (double *)a->Tcur.p;
    L.T_sched = T_sched;
    L.T_base = T_base;
    L.T_value = T;
    if (!L.fuse_rank && (e = launch_rank_merge(keys + kRankMax, keys, K, ord, s)) != hipSuccess)
      return hip_fail(e, "anneal: ranking");
    L.order = ord;
    // the end of this step draws the next one, unless that one re-scores the cell first
    L.draw_next = allow_next && L.fuse_rank && !(a->learn_age == 0 || a->learn_age >= a->refresh);
    if (L.draw_next) {  // with the arguments prepare_next_args uploaded for this configuration
      const int nh = (int)((a->host_step + 1) & 1);
      if (a->nx_ok[nh] && same_next_args(next_args_of(args, a, K, nh), a->nx_host[nh]))
        L.next = (const ProposeArgs *)a->nxargs.p + nh;
      else
        L.draw_next = false;
    }
  }
  a->predrawn = L.draw_next;
  a->predrawn_K = K;
  L.out = reinterpret_cast<StepResult *>(out);
  L.out_base = out_base;
  if ((e = launch_step(L, s)) != hipSuccess) return hip_fail(e, "anneal: evaluation");
  a->host_step += 1;
  if (a->s2) {
    // the S2 rounds read the packed cell itself: nothing else to keep current
  } else if (rec) {
    a->e3_valid = false;
  } else {
    a->rec_valid = false;
    if ((e = launch_ext3_if(a->bits, a->W, a->H, plan->geo, (uint32_t *)a->E3.p,
                            (const int32_t *)a->ksel.p, s)) != hipSuccess)
      return hip_fail(e, "anneal: ext3");
  }
  return LPF_OK;
}

// Uploads (when they changed) the arguments of the next-step draws of a ranked records chain, so
// that a step's end can draw the next step; outside any capture.
lpf_status prepare_next_args(lpf_anneal a, int K, int proposal, const StepLaunch &L, bool rec,
                             hipStream_t s) {
  if (!(proposal == LPF_PROP_LEARNED && a->rank && rec && L.rounds.size() >= 2 &&
        L.rounds[0].C == 64))
    return LPF_OK;
  ProposeArgs none{}, p{};
  lpf_status st = draw_candidates(a, K, proposal, s, nullptr, nullptr, nullptr, 0, 0.0, nullptr,
                                  true, &none, &p, false);
  if (st != LPF_OK) return st;
  bool dirty = false;
  for (int h = 0; h < 2; ++h) {
    const ProposeArgs q = next_args_of(p, a, K, h);
    if (!a->nx_ok[h] || !same_next_args(q, a->nx_host[h])) {
      a->nx_host[h] = q;
      dirty = true;
    }
  }
  if (!dirty) return LPF_OK;
  hipError_t e;
  if ((e = a->nxargs.ensure(2 * sizeof(ProposeArgs))) != hipSuccess ||
      (e = launch_rec_set_next((ProposeArgs *)a->nxargs.p, a->nx_host[0], a->nx_host[1], s)) != hipSuccess)
    return hip_fail(e, "anneal: next-step draw arguments");
  a->nx_ok[0] = a->nx_ok[1] = true;
  return LPF_OK;
}

}  // namespace

lpf_status anneal_step(lpf_anneal a, int K, int proposal, double T, lpf_step_result *out,
                       void *stream) {
  lpf_status st = step_args("anneal_step", a, K, proposal);
  if (st != LPF_OK) return st;
  if (!(T > 0.0)) return fail(LPF_E_INVAL, "anneal_step: T must be > 0");
  if (!out) return fail(LPF_E_INVAL, "anneal_step: out is NULL");
  std::lock_guard<std::mutex> lk(a->ctx->mu);
  DeviceGuard g(a->ctx->dev);
  hipStream_t s = (hipStream_t)stream;
  StepLaunch L;
  DeltaPlan *plan = nullptr;
  bool rec = false;
  if ((st = step_setup(a, K, proposal, s, L, plan, rec)) != LPF_OK) return st;
  // the previous call's end drew this step when it was a ranked step with as many candidates
  if (a->predrawn_K != K || proposal != LPF_PROP_LEARNED) a->predrawn = false;
  if ((st = prepare_next_args(a, K, proposal, L, rec, s)) != LPF_OK) return st;
  return step_enqueue(a, K, proposal, L, plan, rec, nullptr, 0, T, out, -1, s, true);
}

lpf_status lpf_anneal_run(lpf_anneal a, int K, int proposal, const double *T_sched, int nsteps,
                          lpf_step_result *out, void *stream) {
  lpf_status st = step_args("lpf_anneal_run", a, K, proposal);
  if (st != LPF_OK) return st;
  if (nsteps < 0) return fail(LPF_E_INVAL, "lpf_anneal_run: nsteps < 0");
  if (nsteps == 0) return LPF_OK;
  if (!T_sched || !out) return fail(LPF_E_INVAL, "lpf_anneal_run: NULL buffer");
  std::lock_guard<std::mutex> lk(a->ctx->mu);
  DeviceGuard g(a->ctx->dev);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  StepLaunch L;
  DeltaPlan *plan = nullptr;
  bool rec = false;
  if ((st = step_setup(a, K, proposal, s, L, plan, rec)) != LPF_OK) return st;
  const int64_t base = (int64_t)a->host_step;
  int done = 0;
  // runs of kGraphSteps steps as one captured graph, the rest enqueued one by one.  Learned
  // proposals re-score the cell every `refresh` draws (host counter): a graph replays the same
  // pattern when kGraphSteps is a multiple of refresh.
  constexpr int kGraphSteps = 32;
  const bool graphable = proposal != LPF_PROP_LEARNED || kGraphSteps % a->refresh == 0;
  auto age_after = [&](int age, int n) {  // the draw's re-scoring counter after n draws
    for (int i = 0; i < n; ++i) {
      if (age == 0 || age >= a->refresh) age = 0;
      ++age;
    }
    return age;
  };
  a->predrawn = false;
  if ((st = prepare_next_args(a, K, proposal, L, rec, s)) != LPF_OK) return st;
  if (graphable && nsteps >= kGraphSteps) {
    if (!a->cap && (e = hipStreamCreateWithFlags(&a->cap, hipStreamNonBlocking)) != hipSuccess)
      return hip_fail(e, "lpf_anneal_run: capture stream");
    // a ranked chain's steps are drawn by the previous step's end (except those that re-score
    // the cell): the graph's first step is, in every replay after the first, so its draws for
    // the first replay are made here
    if (proposal == LPF_PROP_LEARNED && a->rank && rec && L.rounds.size() >= 2 &&
        L.rounds[0].C == 64 && !(a->learn_age == 0 || a->learn_age >= a->refresh)) {
      if ((st = draw_candidates(a, K, proposal, s, (int64_t *)a->S_acc.p, (StepCtl *)a->ctl.p,
                                T_sched, base, 0.0, (double *)a->Tcur.p, true, nullptr, nullptr,
                                false)) != LPF_OK)
        return st;
      a->predrawn = true;
    }
    // the capture enqueues nothing; the replays run on the caller's stream s
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const uint64_t step_before = a->host_step;
    const bool e3_before = a->e3_valid, rec_before = a->rec_valid, drawn_before = a->predrawn;
    const int age_before = a->learn_age;
    if ((e = hipStreamBeginCapture(a->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
      return hip_fail(e, "lpf_anneal_run: capture");
    lpf_status cst = LPF_OK;
    for (int i = 0; i < kGraphSteps && cst == LPF_OK; ++i)
      cst = step_enqueue(a, K, proposal, L, plan, rec, T_sched, base, 0.0, out, base, a->cap, true);
    hipError_t ce = hipStreamEndCapture(a->cap, &graph);
    // the capture enqueued nothing: restore the host counters it advanced (every replay leaves
    // the next step drawn as the capture found its first: the re-scoring pattern repeats)
    const bool drawn_after = a->predrawn;
    a->host_step = step_before;
    a->e3_valid = e3_before;
    a->rec_valid = rec_before;
    a->learn_age = age_before;
    a->predrawn = drawn_before;
    // (with 32 a multiple of the re-scoring interval they agree; should they not, the steps are
    // enqueued one by one instead)
    const bool replayable = drawn_after == drawn_before;
    if (cst != LPF_OK || ce != hipSuccess ||
        (ce = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0)) != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return cst != LPF_OK ? cst : hip_fail(ce, "lpf_anneal_run: graph");
    }
    for (; replayable && done + kGraphSteps <= nsteps; done += kGraphSteps) {
      if ((e = hipGraphLaunch(exec, s)) != hipSuccess) break;
      a->host_step += kGraphSteps;
      if (proposal == LPF_PROP_LEARNED) a->learn_age = age_after(a->learn_age, kGraphSteps);
      if (!rec && !a->s2) a->rec_valid = false;
      if (rec) a->e3_valid = false;
    }
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return hip_fail(e, "lpf_anneal_run: graph launch");
  }
  for (; done < nsteps; ++done)
    if ((st = step_enqueue(a, K, proposal, L, plan, rec, T_sched, base, 0.0, out, base, s,
                           done + 1 < nsteps)) != LPF_OK)
      return st;
  // a draw made past the run's last step is not used: the next call draws its first step
  a->predrawn = false;
  return LPF_OK;
}

lpf_status lpf_anneal_export(lpf_anneal a, int32_t *pos, int *n1, uint64_t *next_step,
                             void *stream) {
  if (!a) return fail(LPF_E_INVAL, "lpf_anneal_export: state is NULL");
  DeviceGuard g(a->ctx->dev);
  hipStream_t s = (hipStream_t)stream;
  AnnealDev host{};
  hipError_t e;
  if ((e = hipMemcpyAsync(&host, a->dev, sizeof(AnnealDev), hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (pos && (e = hipMemcpyAsync(pos, a->pos, sizeof(int32_t) * (size_t)a->W * a->H,
                                  hipMemcpyDeviceToDevice, s)) != hipSuccess) ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return hip_fail(e, "lpf_anneal_export");
  if (n1) *n1 = host.n1;
  if (next_step) *next_step = host.step;
  return LPF_OK;
}

void lpf_anneal_destroy(lpf_anneal a) {
  if (!a) return;
  {
    DeviceGuard g(a->ctx->dev);
    (void)hipDeviceSynchronize();
    if (a->dev) (void)hipFree(a->dev);
    if (a->pos) (void)hipFree(a->pos);
    a->E3.release();
    a->cand.release();
    a->U.release();
    a->slot.release();
    a->S_acc.release();
    a->ksel.release();
    a->rmeta.release();
    a->rpix.release();
    a->remask.release();
    a->rext.release();
    a->nxargs.release();
    a->rcond.release();
    a->rvbit.release();
    a->rec.release();
    a->ones.release();
    a->dl.release();
    a->ctl.release();
    a->scores.release();
    a->pre.release();
    a->cw1.release();
    a->cw0.release();
    a->cwb.release();
    a->order.release();
    a->rank_buf.release();
    a->S0.release();
    a->eS.release();
    a->eCtl.release();
    a->Tcur.release();
    if (a->cap) (void)hipStreamDestroy(a->cap);
  }
  delete a;
}

lpf_status lpf_batch(lpf_ctx c, const uint64_t *bits_pool, const lpf_image_desc *descs,
                     int n_images, unsigned phase_mask, int out_layout, uint32_t *counts_pool,
                     void *stream) {
  if (!c) return fail(LPF_E_INVAL, "lpf_batch: ctx is NULL");
  if (n_images < 0 || n_images > 65535) return fail(LPF_E_INVAL, "lpf_batch: n_images outside [0, 65535]");
  if (n_images == 0) return LPF_OK;
  if (!bits_pool || !descs || !counts_pool) return fail(LPF_E_INVAL, "lpf_batch: NULL buffer");
  if (phase_mask < 1 || phase_mask > 3) return fail(LPF_E_INVAL, "lpf_batch: phase_mask");
  if (out_layout != LPF_OUT_HALF && out_layout != LPF_OUT_GRID)
    return fail(LPF_E_INVAL, "lpf_batch: out_layout");
  for (int i = 0; i < n_images; ++i) {
    const lpf_image_desc &d = descs[i];
    lpf_status st = check_image_args("lpf_batch", d.W, d.H, d.cx, d.cy, phase_mask);
    if (st != LPF_OK) return fail(st, std::string(lpf_last_error()) + " (image " + std::to_string(i) + ")");
    if (d.bits_off < 0 || d.counts_off < 0)
      return fail(LPF_E_INVAL, "lpf_batch: negative offset (image " + std::to_string(i) + ")");
  }
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->dev);
  if (!g.ok) return fail(LPF_E_DEVICE, "lpf_batch: cannot select the context's device");
  hipStream_t s = (hipStream_t)stream;
  // cache key: layout, shape overrides and every descriptor (the buffers are set per call)
  std::string key;
  {
    char buf[96];
    snprintf(buf, sizeof buf, "%u|%d|%d|%d|%d|%d|%d|", phase_mask, out_layout, n_images,
             c->force_R, c->force_S, c->force_wpg, c->force_lds);
    key = buf;
    key.append(reinterpret_cast<const char *>(descs), sizeof(lpf_image_desc) * (size_t)n_images);
  }
  auto it = c->batch_graphs.find(key);
  if (it == c->batch_graphs.end() && c->batch_graphs.size() >= kMaxBatchGraphs) {
    auto lru = c->batch_graphs.begin();
    for (auto j = c->batch_graphs.begin(); j != c->batch_graphs.end(); ++j)
      if (j->second->last_use < lru->second->last_use) lru = j;
    (void)hipDeviceSynchronize();  // its last replay may still run on any stream
    free_batch_graph(lru->second);
    c->batch_graphs.erase(lru);
  }
  if (it == c->batch_graphs.end()) {
    // 8 waves per group, or 16 when some image's rows need so much LDS that only one group fits
    // a CU (four waves per SIMD either way; one launch has one group size); every image's shape
    // is checked while its plan is built
    int wpg = 8;
    std::vector<FullImg> imgs(n_images);
    std::vector<int64_t> bits_off(n_images), ext_off(n_images), counts_off(n_images);
    std::vector<std::pair<int64_t, int2>> items;
    int64_t ext_total = 0;
    size_t stage_max = 0;
    bool any_tiled = false;
    int max_we = 1, max_h = 1;
    for (int pass = 0; pass < 2; ++pass) {
    items.clear();
    ext_total = 0;
    stage_max = 0;
    any_tiled = false;
    max_we = 1;
    max_h = 1;
    for (int i = 0; i < n_images; ++i) {
      const lpf_image_desc &d = descs[i];
      FullPlan *plan = nullptr;
      const int saved_wpg = c->force_wpg;
      c->force_wpg = wpg;
      lpf_status st = get_full_plan(c, d.W, d.H, d.cx, d.cy, plan);
      c->force_wpg = saved_wpg;
      if (st != LPF_OK) return st;
      const FullShape &sh = plan->sh;
      ext_off[i] = ext_total;
      bits_off[i] = d.bits_off;
      ext_total += (int64_t)(sh.glob ? sh.lds_rows : d.H) * sh.we;
      imgs[i] = make_img(*plan, nullptr, nullptr, d.W, d.H, d.cx, d.cy, out_layout);
      counts_off[i] = d.counts_off;
      if (!sh.glob) stage_max = std::max(stage_max, (size_t)sh.lds_rows * sh.rst);
      any_tiled = any_tiled || sh.ntiles > 1;
      max_we = std::max(max_we, sh.we);
      max_h = std::max(max_h, sh.glob ? sh.lds_rows : d.H);
      const int64_t rows_work = (int64_t)d.H * sh.S;
      for (int b = 0; b < sh.nbins; ++b)
        items.push_back({plan->bin_cost[b] * rows_work * sh.R + (int64_t)sh.lds_rows * sh.we * sh.ntiles,
                         make_int2(i, b)});
    }
    if (pass == 0 && (stage_max * 4 + (size_t)kSlotWords * 4) * 2 > (size_t)kMaxLds) {
      wpg = 16;
      continue;
    }
    break;
    }
    std::stable_sort(items.begin(), items.end(),
                     [](const std::pair<int64_t, int2> &a, const std::pair<int64_t, int2> &b) {
                       return a.first > b.first;
                     });
    std::vector<int2> item_list(items.size());
    for (size_t k = 0; k < items.size(); ++k) item_list[k] = items[k].second;
    const size_t lds_bytes = stage_max * 4 + (size_t)kSlotWords * 4;
    (void)any_tiled;
    if (lds_bytes > (size_t)(kMaxLds - kBatchStaticLds))
      return fail(LPF_E_UNSUPPORTED, "lpf_batch: staging exceeds LDS");
    BatchGraph *b = new (std::nothrow) BatchGraph();
    if (!b) return fail(LPF_E_NOMEM, "lpf_batch: host memory");
    hipError_t e;
    if ((e = hipMalloc(&b->ext, sizeof(uint32_t) * (size_t)std::max<int64_t>(ext_total, 1))) != hipSuccess ||
        (e = hipMalloc(&b->imgs, sizeof(FullImg) * n_images)) != hipSuccess ||
        (e = hipMalloc(&b->args, sizeof(BatchArgs))) != hipSuccess ||
        (e = hipMalloc(&b->counts_off, sizeof(int64_t) * n_images)) != hipSuccess ||
        (e = hipMalloc(&b->items, sizeof(int2) * item_list.size())) != hipSuccess ||
        (e = hipMalloc(&b->bits_off, sizeof(int64_t) * n_images)) != hipSuccess ||
        (e = hipMalloc(&b->ext_off, sizeof(int64_t) * n_images)) != hipSuccess ||
        (e = hipMalloc(&b->counter, sizeof(int))) != hipSuccess) {
      free_batch_graph(b);
      return hip_fail(e, "lpf_batch: allocation");
    }
    for (int i = 0; i < n_images; ++i) imgs[i].E = b->ext + ext_off[i];
    if ((e = hipMemcpy(b->imgs, imgs.data(), sizeof(FullImg) * n_images, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(b->items, item_list.data(), sizeof(int2) * item_list.size(), hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(b->bits_off, bits_off.data(), sizeof(int64_t) * n_images, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(b->ext_off, ext_off.data(), sizeof(int64_t) * n_images, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(b->counts_off, counts_off.data(), sizeof(int64_t) * n_images, hipMemcpyHostToDevice)) != hipSuccess) {
      free_batch_graph(b);
      return hip_fail(e, "lpf_batch: upload");
    }
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->dev);
    const int per_cu = std::max<int>(1, std::min<int>(4, (int)(kMaxLds / std::max<size_t>(lds_bytes, 1))));
    b->n_items = (int)item_list.size();
    b->n_wg = std::max(1, std::min(b->n_items, cus * per_cu));
    // capture on a private stream, launch on the caller's
    hipStream_t cap;
    if ((e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking)) != hipSuccess) {
      free_batch_graph(b);
      return hip_fail(e, "lpf_batch: capture stream");
    }
    hipError_t ce = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (ce == hipSuccess) {
      hipError_t e1 = launch_ext_batch(b->imgs, n_images, max_we, max_h, b->args, b->bits_off,
                                       b->ext, b->ext_off, cap);
      hipError_t e2 = launch_batch(b->imgs, b->args, b->counts_off, b->items, b->n_items,
                                   b->counter, wpg, phase_mask, lds_bytes, (int)stage_max,
                                   b->n_wg, cap);
      ce = hipStreamEndCapture(cap, &b->graph);
      if (ce == hipSuccess && (e1 != hipSuccess || e2 != hipSuccess)) ce = e1 != hipSuccess ? e1 : e2;
    }
    if (ce == hipSuccess) ce = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cap);
    if (ce != hipSuccess) {
      free_batch_graph(b);
      return hip_fail(ce, "lpf_batch: graph capture");
    }
    it = c->batch_graphs.emplace(key, b).first;
  }
  it->second->last_use = ++c->batch_clock;
  hipError_t e = launch_batch_args(it->second->args, bits_pool, counts_pool, s);
  if (e != hipSuccess) return hip_fail(e, "lpf_batch: buffers");
  e = hipGraphLaunch(it->second->exec, s);
  if (e != hipSuccess) return hip_fail(e, "lpf_batch: graph launch");
  return LPF_OK;
}

lpf_status lpf_autotune_full(lpf_ctx c, const uint64_t *bits, int W, int H, int cx, int cy,
                             unsigned phase_mask, void *stream, double *best_ms) {
  if (!c) return fail(LPF_E_INVAL, "lpf_autotune_full: ctx is NULL");
  lpf_status st = check_image_args("lpf_autotune_full", W, H, cx, cy, phase_mask);
  if (st != LPF_OK) return st;
  if (!bits) return fail(LPF_E_INVAL, "lpf_autotune_full: bits is NULL");
  hipStream_t s = (hipStream_t)stream;
  const int64_t nv = lpf_num_vectors(cx, cy);
  const int nph = nph_of(phase_mask);
  uint32_t *tmp = nullptr;
  hipError_t e;
  {
    DeviceGuard g(c->dev);
    if ((e = hipMalloc(&tmp, sizeof(uint32_t) * (size_t)nph * nv)) != hipSuccess)
      return hip_fail(e, "lpf_autotune_full: allocation");
  }
  const int saved[4] = {c->force_R, c->force_S, c->force_wpg, c->force_lds};
  {
    std::lock_guard<std::mutex> lk(c->mu);
    c->tuned.erase(std::make_tuple(W, H, cx, cy));
  }
  TunedShape best{};
  best.ms = 1e30;
  const int swd = (W + 31) / 32;
  hipEvent_t e0, e1;
  {
    DeviceGuard g(c->dev);
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
  }
  for (int R : {2, 4, 8, 16}) {
    if (R > 2 * next_pow2(swd) && R > 2) continue;
    for (int wpg : {4, 8, 16}) {
      for (int lds : {64 * 1024, kBigLds}) {
        if (wpg == 16 && lds != kBigLds) continue;  // 16 waves only at one group per CU
        c->force_R = R;
        c->force_S = 0;
        c->force_wpg = wpg;
        c->force_lds = lds;
        float ms_best = 1e30f;
        bool ok = true;
        for (int rep = 0; rep < 3 && ok; ++rep) {
          DeviceGuard g(c->dev);
          (void)hipEventRecord(e0, s);
          ok = lpf_full(c, bits, W, H, cx, cy, phase_mask, LPF_OUT_HALF, tmp, stream) == LPF_OK;
          (void)hipEventRecord(e1, s);
          if (ok && hipEventSynchronize(e1) == hipSuccess) {
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (rep) ms_best = std::min(ms_best, ms);  // first run builds the plan
          }
        }
        if (ok && ms_best < best.ms) {
          best.R = R;
          best.wpg = wpg;
          best.lds = lds;
          best.ms = ms_best;
        }
      }
    }
  }
  c->force_R = saved[0];
  c->force_S = saved[1];
  c->force_wpg = saved[2];
  c->force_lds = saved[3];
  {
    DeviceGuard g(c->dev);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(tmp);
  }
  if (best.ms >= 1e29) return fail(LPF_E_UNSUPPORTED, "lpf_autotune_full: no shape ran");
  {
    std::lock_guard<std::mutex> lk(c->mu);
    c->tuned[std::make_tuple(W, H, cx, cy)] = best;
  }
  if (best_ms) *best_ms = best.ms;
  return LPF_OK;
}

lpf_status lpf_get_tuned_shape(lpf_ctx c, int W, int H, int cx, int cy, int *R, int *wpg,
                               int *lds_bytes) {
  if (!c) return fail(LPF_E_INVAL, "lpf_get_tuned_shape: ctx is NULL");
  std::lock_guard<std::mutex> lk(c->mu);
  auto it = c->tuned.find(std::make_tuple(W, H, cx, cy));
  if (it == c->tuned.end()) return fail(LPF_E_INVAL, "lpf_get_tuned_shape: not tuned");
  if (R) *R = it->second.R;
  if (wpg) *wpg = it->second.wpg;
  if (lds_bytes) *lds_bytes = it->second.lds;
  return LPF_OK;
}

lpf_status lpf_cnn_create(lpf_ctx c, int W, int H, int max_batch, int max_samples,
                          const float *params, lpf_cnn *out, void *stream) {
  if (!out) return fail(LPF_E_INVAL, "lpf_cnn_create: out is NULL");
  *out = nullptr;
  if (!c) return fail(LPF_E_INVAL, "lpf_cnn_create: ctx is NULL");
  if (W < 1 || H < 1 || W > 65535 || H > 65535 || max_batch < 1 || max_samples < 1 ||
      (int64_t)W * H * max_batch > ((int64_t)1 << 28) || max_samples > (1 << 26))
    return fail(LPF_E_INVAL, "lpf_cnn_create: sizes");
  lpf_cnn n = new (std::nothrow) lpf_cnn_s();
  if (!n) return fail(LPF_E_NOMEM, "lpf_cnn_create: host memory");
  n->ctx = c;
  n->W = W;
  n->H = H;
  n->max_batch = max_batch;
  n->max_samples = max_samples;
  DeviceGuard g(c->dev);
  const int64_t np = (int64_t)W * H * max_batch;
  const int64_t cb = cnn_conv_blocks(np), hb = (np + 255) / 256;
  hipError_t e = hipSuccess;
  auto get = [&](void **p, size_t bytes) {
    if (e != hipSuccess) return;
    e = hipMalloc(p, std::max<size_t>(bytes, 16));
    if (e == hipSuccess) n->allocs.push_back(*p);
  };
  CnnBufs &B = n->b;
  get((void **)&B.prm, 4 * kCnnParams);
  get((void **)&B.mom, 4 * kCnnParams);
  get((void **)&B.vel, 4 * kCnnParams);
  get((void **)&B.Wf, 2 * 3 * 2304);
  get((void **)&B.Wt, 2 * 3 * 2304);
  get((void **)&B.W4bf, 4 * 16);
  get((void **)&B.X0, 2 * 4 * (size_t)np);
  get((void **)&B.A1, 2 * 16 * (size_t)np);
  get((void **)&B.A2, 2 * 16 * (size_t)np);
  get((void **)&B.A3, 2 * 16 * (size_t)np);
  get((void **)&B.dZ1, 2 * 16 * (size_t)np);
  get((void **)&B.dZ2, 2 * 16 * (size_t)np);
  get((void **)&B.dZ3, 2 * 16 * (size_t)np);
  get((void **)&B.S, 4 * (size_t)np);
  get((void **)&B.r, 4 * (size_t)max_samples);
  get((void **)&B.dS, 8 * (size_t)np);
  get((void **)&B.part1, 4 * (size_t)cb * (9 * 256 + 16));
  get((void **)&B.part2, 4 * (size_t)cb * (9 * 256 + 16));
  get((void **)&B.part3, 4 * (size_t)cb * (9 * 256 + 16));
  get((void **)&B.part_h, 4 * (size_t)hb * 17);
  get((void **)&B.slices, 4 * (size_t)64 * kCnnParams);
  hipStream_t s = (hipStream_t)stream;
  if (e == hipSuccess) {
    if (params) e = hipMemcpyAsync(B.prm, params, 4 * kCnnParams, hipMemcpyDeviceToDevice, s);
    else e = hipMemsetAsync(B.prm, 0, 4 * kCnnParams, s);
  }
  if (e == hipSuccess) e = hipMemsetAsync(B.mom, 0, 4 * kCnnParams, s);
  if (e == hipSuccess) e = hipMemsetAsync(B.vel, 0, 4 * kCnnParams, s);
  if (e == hipSuccess) e = cnn_pack(B, s);
  if (e != hipSuccess) {
    lpf_cnn_destroy(n);
    return hip_fail(e, "lpf_cnn_create");
  }
  *out = n;
  return LPF_OK;
}

lpf_status lpf_cnn_set_params(lpf_cnn n, const float *params, void *stream) {
  if (!n || !params) return fail(LPF_E_INVAL, "lpf_cnn_set_params: NULL argument");
  DeviceGuard g(n->ctx->dev);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(n->b.prm, params, 4 * kCnnParams, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(n->b.mom, 0, 4 * kCnnParams, s);
  if (e == hipSuccess) e = hipMemsetAsync(n->b.vel, 0, 4 * kCnnParams, s);
  if (e == hipSuccess) e = cnn_pack(n->b, s);
  return e == hipSuccess ? LPF_OK : hip_fail(e, "lpf_cnn_set_params");
}

lpf_status lpf_cnn_get_params(lpf_cnn n, float *params, void *stream) {
  if (!n || !params) return fail(LPF_E_INVAL, "lpf_cnn_get_params: NULL argument");
  DeviceGuard g(n->ctx->dev);
  hipError_t e = hipMemcpyAsync(params, n->b.prm, 4 * kCnnParams, hipMemcpyDeviceToDevice,
                                (hipStream_t)stream);
  return e == hipSuccess ? LPF_OK : hip_fail(e, "lpf_cnn_get_params");
}

lpf_status lpf_cnn_forward(lpf_cnn n, const uint64_t *bits, int batch, float *scores,
                           void *stream) {
  if (!n || !bits || !scores) return fail(LPF_E_INVAL, "lpf_cnn_forward: NULL argument");
  if (batch < 1 || batch > n->max_batch) return fail(LPF_E_INVAL, "lpf_cnn_forward: batch");
  DeviceGuard g(n->ctx->dev);
  // one image: the single-launch kernel (same scores, bit for bit)
  hipError_t e = batch == 1 ? cnn_score(n->b, bits, n->W, n->H, scores, (hipStream_t)stream)
                            : cnn_forward(n->b, bits, n->W, n->H, batch, scores, (hipStream_t)stream);
  return e == hipSuccess ? LPF_OK : hip_fail(e, "lpf_cnn_forward");
}

lpf_status lpf_cnn_grad(lpf_cnn n, const uint64_t *bits, int batch, const lpf_cnn_sample *samples,
                        int ns, float *grad, float *loss, void *stream) {
  if (!n || !bits || !samples || !grad || !loss) return fail(LPF_E_INVAL, "lpf_cnn_grad: NULL argument");
  if (batch < 1 || batch > n->max_batch) return fail(LPF_E_INVAL, "lpf_cnn_grad: batch");
  if (ns < 1 || ns > n->max_samples) return fail(LPF_E_INVAL, "lpf_cnn_grad: n");
  DeviceGuard g(n->ctx->dev);
  hipError_t e = cnn_grad(n->b, bits, n->W, n->H, batch,
                          reinterpret_cast<const CnnSample *>(samples), ns, grad, loss,
                          (hipStream_t)stream);
  return e == hipSuccess ? LPF_OK : hip_fail(e, "lpf_cnn_grad");
}

lpf_status lpf_cnn_adam(lpf_cnn n, const float *grad, int t, float lr, float beta1, float beta2,
                        float eps, void *stream) {
  if (!n || !grad) return fail(LPF_E_INVAL, "lpf_cnn_adam: NULL argument");
  if (t < 1 || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return fail(LPF_E_INVAL, "lpf_cnn_adam: t >= 1, lr > 0, 0 <= beta < 1, eps > 0");
  DeviceGuard g(n->ctx->dev);
  const float c1 = (float)(1.0 - std::pow((double)beta1, (double)t));
  const float c2 = (float)(1.0 - std::pow((double)beta2, (double)t));
  hipError_t e = cnn_adam(n->b, grad, lr, beta1, beta2, eps, c1, c2, (hipStream_t)stream);
  return e == hipSuccess ? LPF_OK : hip_fail(e, "lpf_cnn_adam");
}

void lpf_cnn_destroy(lpf_cnn n) {
  if (!n) return;
  {
    DeviceGuard g(n->ctx->dev);
    (void)hipDeviceSynchronize();
    for (void *p : n->allocs) (void)hipFree(p);
  }
  delete n;
}

lpf_status lpf_anneal_set_proposal(lpf_anneal a, lpf_cnn net, const float *scores, float beta,
                                   float eps_uniform, int refresh, int rank) {
  if (!a) return fail(LPF_E_INVAL, "lpf_anneal_set_proposal: state is NULL");
  if (net && (net->W != a->W || net->H != a->H))
    return fail(LPF_E_INVAL, "lpf_anneal_set_proposal: network built for another cell size");
  if (!(beta >= 0.f) || !(eps_uniform >= 0.f && eps_uniform <= 1.f))
    return fail(LPF_E_INVAL, "lpf_anneal_set_proposal: beta >= 0, 0 <= eps_uniform <= 1");
  if (refresh < 1) return fail(LPF_E_INVAL, "lpf_anneal_set_proposal: refresh >= 1");
  if (rank != 0 && rank != 1) return fail(LPF_E_INVAL, "lpf_anneal_set_proposal: rank is 0 or 1");
  a->refresh = refresh;
  a->rank = rank != 0;
  a->learn_age = 0;
  a->predrawn = false;
  a->net = net;
  a->scores_ext = net ? nullptr : scores;
  a->beta = beta;
  a->eps = eps_uniform;
  return LPF_OK;
}

lpf_status lpf_rank(lpf_ctx c, const int32_t *cand, const float *score, int K, int32_t *order,
                    void *stream) {
  if (!c) return fail(LPF_E_INVAL, "lpf_rank: ctx is NULL");
  if (K < 1 || K > (1 << 20)) return fail(LPF_E_INVAL, "lpf_rank: K outside [1, 2^20]");
  if (!cand || !score || !order) return fail(LPF_E_INVAL, "lpf_rank: NULL buffer");
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->dev);
  if (!g.ok) return fail(LPF_E_DEVICE, "lpf_rank: cannot select the context's device");
  hipError_t e = c->rank_buf.ensure(kRankScratch);
  if (e != hipSuccess) return hip_fail(e, "lpf_rank: scratch");
  uint64_t *keys = (uint64_t *)c->rank_buf.p;
  e = launch_rank(reinterpret_cast<const int2 *>(cand), score, K, order, keys, keys + kRankMax,
                  (hipStream_t)stream);
  return e == hipSuccess ? LPF_OK : hip_fail(e, "lpf_rank");
}

lpf_status lpf_anneal_propose(lpf_anneal a, int K, int proposal, int32_t *cand_out, void *stream) {
  if (!a || !cand_out) return fail(LPF_E_INVAL, "lpf_anneal_propose: NULL argument");
  if (K < 1 || K > (1 << 20)) return fail(LPF_E_INVAL, "lpf_anneal_propose: K");
  if (proposal < LPF_PROP_UNIFORM || proposal > LPF_PROP_LEARNED)
    return fail(LPF_E_INVAL, "lpf_anneal_propose: proposal");
  if (proposal == LPF_PROP_LEARNED && !a->net && !a->scores_ext)
    return fail(LPF_E_INVAL, "lpf_anneal_propose: learned proposal without lpf_anneal_set_proposal");
  std::lock_guard<std::mutex> lk(a->ctx->mu);
  DeviceGuard g(a->ctx->dev);
  hipStream_t s = (hipStream_t)stream;
  a->predrawn = false;  // this draw overwrites the half a draw made ahead would be in
  lpf_status st = draw_candidates(a, K, proposal, s);
  if (st != LPF_OK) return st;
  const size_t half = (size_t)(a->host_step & 1) * (size_t)K;
  hipError_t e = launch_copy_cand((const int2 *)a->cand.p + half, K, cand_out, s);
  return e == hipSuccess ? LPF_OK : hip_fail(e, "lpf_anneal_propose");
}

lpf_status lpf_anneal_delta_energy(lpf_anneal a, const int32_t *swaps, int n, double *de,
                                   void *stream) {
  if (!a || (n > 0 && (!swaps || !de))) return fail(LPF_E_INVAL, "lpf_anneal_delta_energy: NULL argument");
  if (n < 0 || n > (1 << 20)) return fail(LPF_E_INVAL, "lpf_anneal_delta_energy: n");
  if (n == 0) return LPF_OK;
  lpf_ctx c = a->ctx;
  std::lock_guard<std::mutex> lk(c->mu);
  DeviceGuard g(c->dev);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  const bool rec = !a->s2 && use_records(a);
  StepLaunch L{};
  L.s2 = a->s2;
  L.records = rec;
  L.rounds = step_rounds(n, false);
  DeltaPlan *plan = nullptr;
  lpf_status st;
  if (a->s2) {
    S2Plan *sp = nullptr;
    if ((st = get_s2_plan(c, a->W, a->H, a->cx, a->cy, sp)) != LPF_OK) return st;
    L.s2vec = sp->vec;
    L.use_lds = s2_img_lds(a->W, a->H);
    s2_rounds(L.rounds, sp->nv);
  } else if (rec) {
    if ((st = setup_records(a, s)) != LPF_OK) return st;
    records_rounds(L.rounds);
  } else {
    if ((st = recount_rounds(a, L.rounds, plan)) != LPF_OK) return st;
    if ((st = prepare_eval(a, false, plan->geo, s)) != LPF_OK) return st;
    L.E = (const uint32_t *)a->E3.p;
    L.geo = plan->geo;
    L.runs = plan->runs;
    L.use_lds = plan->use_lds;
  }
  if ((e = a->eS.ensure(sizeof(int64_t) * (size_t)n)) != hipSuccess ||
      (e = a->eCtl.ensure(sizeof(StepCtl))) != hipSuccess)
    return hip_fail(e, "lpf_anneal_delta_energy: scratch");
  L.rg = a->rg;
  L.bits = a->bits;
  L.W = a->W;
  L.H = a->H;
  L.cand = reinterpret_cast<const int2 *>(swaps);
  L.K = n;
  L.phase_mask = a->mask;
  L.nv = (int)lpf_num_vectors(a->cx, a->cy);
  L.counts = a->counts;
  L.target = a->target;
  L.N = a->Neff;
  L.Nt = a->Nt;
  L.S_acc = (int64_t *)a->eS.p;
  L.ctl = (StepCtl *)a->eCtl.p;
  e = launch_energy(L, de, s);
  return e == hipSuccess ? LPF_OK : hip_fail(e, "lpf_anneal_delta_energy");
}

lpf_status lpf_anneal_set_method(lpf_anneal a, int method) {
  if (!a) return fail(LPF_E_INVAL, "lpf_anneal_set_method: state is NULL");
  if (method != LPF_DELTA_AUTO && method != LPF_DELTA_RECOUNT && method != LPF_DELTA_RECORDS)
    return fail(LPF_E_INVAL, "lpf_anneal_set_method: method");
  if (a->s2 && method != LPF_DELTA_AUTO)
    return fail(LPF_E_UNSUPPORTED, "lpf_anneal_set_method: an S2 chain has a single method");
  if (a->sample && method == LPF_DELTA_RECOUNT)
    return fail(LPF_E_UNSUPPORTED, "lpf_anneal_set_method: a sampled chain uses the records");
  std::string why;
  if (method == LPF_DELTA_RECORDS && !records_fit(a, nullptr, &why))
    return fail(LPF_E_UNSUPPORTED, "lpf_anneal_set_method: records: " + why);
  std::lock_guard<std::mutex> lk(a->ctx->mu);
  a->method = method;
  a->predrawn = false;
  a->rec_choice = a->sample ? 1 : -1;
  return LPF_OK;
}

int lpf_anneal_get_method(lpf_anneal a) {
  if (!a) {
    fail(LPF_E_INVAL, "lpf_anneal_get_method: state is NULL");
    return -1;
  }
  if (a->s2) return LPF_DELTA_S2;
  std::lock_guard<std::mutex> lk(a->ctx->mu);
  DeviceGuard g(a->ctx->dev);
  return use_records(a) ? LPF_DELTA_RECORDS : LPF_DELTA_RECOUNT;
}

}  // extern "C"
