// Internal declarations shared by the HIP sources of liblpf (not part of the C ABI).
#pragma once

#include <algorithm>
#include <vector>

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lpf {

// A vector of D_c and its canonical index.
struct VecDesc {
  int16_t dx, dy;
  int32_t idx;
};

// A chain of the full-evaluation plan: the walked vector (dx, dy), its members
// mems[m0 .. m0 + nm) in increasing l, and lw = the last member's l (the walked vector itself).
struct ChainDesc {
  int16_t dx, dy;
  int32_t m0, nm, lw;
};
// A member of a chain: vector (dx, dy) with canonical index idx, whose path is (up to a
// translation) pixels 0..l of the chain's walked path.
struct MemDesc {
  int32_t idx;
  int16_t dx, dy;
  int32_t l;
};

// Tile shape of the full-evaluation kernel.
//   R       consecutive 32-pixel words of one row owned by a lane
//   S       lanes per image row (R*S >= ceil(W/32)); a wave covers 64/S rows per band
//   wpg     waves per workgroup
//   tile    start rows per workgroup (row tile); ntiles = ceil(H / tile)
//   rst     LDS row stride in dwords (>= we), chosen against bank conflicts
//   we      dwords per row of the extended image: S*R + (cx >> 5) + 1
//   lds_rows rows staged in LDS per workgroup: tile + cy + 64/S
//   nwb     waves sharing a chain (each takes every nwb-th band of a tile); wpg / nwb chain groups
//   nbins   workgroup-level bins of chains (one workgroup each)
//   glob    1: the halo rows do not fit in LDS; rows are read from the extended image in device
//           memory (lds_rows rows of E, periodic), one tile of H rows, only count slots in LDS
struct FullShape {
  int R, S, wpg, tile, ntiles, rst, we, lds_rows;
  int nwb;
  int nbins;
  int glob;
};

// Count slots of one bin in LDS (two words per member): at most kSlotWords / 2 members per bin.
constexpr int kSlotWords = 512;
// LDS the persistent batch kernel keeps for itself (the claimed work item), below the 160 KiB.
constexpr int kBatchStaticLds = 256;

// One image as seen by the full-evaluation kernels.
struct FullImg {
  const uint32_t *E;          // extended image, H x we dwords
  uint32_t *out;              // counts in the output layout
  const ChainDesc *chains;    // chains in bin order
  const MemDesc *mems;        // members in chain order
  const int32_t *bin_off;     // nbins + 1 (chain offsets)
  int W, H, cx, cy, R, S, we, rst, tile, ntiles, lds_rows, nv, layout, nbins, nwb, glob;
  // Monte-Carlo position set: extended rows of its mask like E (bit j of row y = position
  // (j mod W, y) is counted), sample_stride = we dwords per row; nullptr = every pixel
  const uint32_t *sample;
  int sample_stride;
};

// Chains of the canonical half domain D_c (plan_full.hip): every vector in exactly one chain.
struct ChainSet {
  std::vector<ChainDesc> chains;  // m0 indexes mems
  std::vector<MemDesc> mems;
  int64_t walk = 0;               // sum over chains of (lw + 1): pixels walked per start word
  int64_t path_pixels = 0;        // M_c = sum over D_c of (n + 1)
};
void build_chains(int cx, int cy, ChainSet &out);
// Chains cut into pieces of at most kSlotWords / 4 members and packed into bins (one workgroup
// each), longest processing time first: chains in bin order with their members (m0 indexes
// mems), off[nbins + 1] chain offsets, cost = pixels walked + 3 per member of each bin.
struct BinPlan {
  std::vector<ChainDesc> chains;
  std::vector<MemDesc> mems;
  std::vector<int32_t> off;
  std::vector<int64_t> cost;
  int nbins = 0;
};
void pack_bins(const ChainSet &all, int64_t nb_want, BinPlan &out);

// Geometry of one extended image used by the delta kernel (see k_delta.hip): width, height,
// dwords per row, dword offset in the concatenated buffer, and the 64-bit pattern of columns
// 0, W, 2W, ... (1 when W >= 64).
struct ImgGeo {
  int W, H, we, off;
  uint64_t pat;
};
struct DeltaGeo {
  ImgGeo g[3];  // image, transposed image, anti-transposed image
  int total;    // dwords of all three
  int hy;       // halo rows below each image
};
// A vector of the delta plan: minor extent m of its flat form, canonical index, image frame,
// offset of its m+1 runs (alpha | beta << 16, normalised columns) in the run table.
struct DeltaVec {
  int32_t m, idx, img, run_off;
};
struct DeltaLaunch {
  const uint32_t *E;
  DeltaGeo geo;
  const uint64_t *bits;
  int W, H;
  const int2 *cand;
  int K;
  const DeltaVec *vecs;
  const int32_t *chunk_off;
  const uint32_t *runs;
  unsigned phase_mask;
  int nv;
  int32_t *delta_out;
  int nchunks;
  bool use_lds;
};

// ---- stateless interchange deltas by offset rows (k_delta.hip, plan_delta.hip) ----
// For placement s - p_k of a vector with major extent n and minor extent m, its pixel with path
// index i = k + d is s + (p_{k+d} - p_k): the major coordinate moves by d (times the row step sr)
// and the minor one by y_{k+d} - y_k, which is floor(d m / n) or one more for every k (y_k the
// digitised minor coordinate of eq. (segments)).  So for a fixed d the pixels of all placements
// k lie on one frame row at two neighbouring minor offsets, and one 32-bit window of that row,
// two single-bit extracts and a select give the pixel word of all (up to 32) placements at once.
// Vectors of one class (frame, row step, minor sign, n) with consecutive m share the d loop and
// the window.
constexpr int kDiagG = 16;
// Every field is a 32-bit word: the kernel reads them with scalar loads (sub-dword fields would
// be read per lane).
struct DiagGroup {
  int32_t row0;         // first row of block 0
  int32_t boff[9];      // rows of placement block b: row0 + boff[b] .. row0 + boff[b + 1] - 1
  int32_t idx[kDiagG];  // canonical vector indices
  int32_t n;            // major extent
  int32_t G;            // vectors
  int32_t frame;        // 0: frame rows are y (steep vectors), 1: rows are x (flat vectors)
  int32_t sr;           // frame row step per unit of d (+1 or -1)
  int32_t nb;           // placement blocks of 32 (n + 1 placements)
  int32_t pad;
};
struct DiagRow {
  int32_t d;                  // path index minus placement index (never 0)
  int32_t o;                  // window origin: minor offset (from the lane's pixel) of window bit 0
  uint32_t valid;             // placements t of the block whose pixel index k + d lies in [0, n]
  uint32_t hs[kDiagG];        // bit t set: placement t's pixel is window bit j + 1, else bit j
  uint32_t jp[kDiagG / 4];    // byte g % 4 of word g / 4: window bit j of the lower of vector
                              // g's two offsets (<= 30)
  uint32_t pad;
};
// Two extended frames with periodic halos: frame 0 rows r = y + cy (bits along x), frame 1 rows
// r = x + cx (bits along y); bit B[f] + u of a row is minor coordinate u (mod the period).
struct DiagGeo {
  int we[2];        // dwords per row
  int rows[2];      // rows per frame
  int off[2];       // first dword of each frame
  int total;        // dwords of both frames
  int B[2];         // bit of minor coordinate 0
  int rowoff[2];    // row of major coordinate 0 (cy, cx)
  uint32_t pat[2];  // bits 0, P, 2P, ... below 32 for the minor period P (W, H)
};
struct DiagTable {
  std::vector<DiagGroup> groups;  // chunk order
  std::vector<DiagRow> rows;
  std::vector<int32_t> chunk_off;  // nchunks + 1
};
struct DiagLaunch {
  const uint32_t *F;
  DiagGeo geo;
  const uint64_t *bits;
  int W, H;
  const int2 *cand;
  int K;
  const DiagGroup *groups;
  const int32_t *chunk_off;
  const DiagRow *rows;
  int nchunks;
  unsigned phase_mask;
  int nv;
  int32_t *delta_out;
  bool use_lds;
};

// Per-step control block of the round-wise evaluation (k_step.hip).
struct alignas(16) StepCtl {
  int32_t done;      // a round has accepted
  int32_t ks;        // accepted candidate, -1 when none
  int32_t a, b;      // its interchange (cand[ks]), set with ks, so that one load gives all three
  long long S;       // its integer energy sum
  uint64_t next_step;  // ranked records steps: the step after this one (set by the step's round 0)
};

// One round of candidates k0 .. k0 + C - 1.  Recount method: `block` candidates per workgroup
// and the vector chunking used (plan arrays); records method: vectors per workgroup.
struct RoundPlan {
  int k0, C, block, nchunks;
  int pi0, pC;  // the previous round, decided at the start of this one (pC = 0: none)
  const DeltaVec *vecs;
  const int32_t *chunk_off;
};

// Placement-state records of an annealing chain (k_rec.hip).  For vector v (canonical order)
// and placement x, ones(v, x) counts the phase-1 pixels on x + path(v).  The record of pixel q
// holds, for every v and every path index k, the state of placement q - p_k: plane A (read for
// the pixel leaving phase 1) = [ones == 1] (phase 0) and [ones == n+1] (phase 1); plane B (read
// for the pixel entering phase 1) = [ones == 0] and [ones == n].  Bit j = off(v) + k.
struct RecGeo {
  int nv, Mc, Rw, nph;  // vectors, path pixels in total, dwords per plane, phases kept
  int W, H;
  int64_t rstride;      // dwords per pixel record = 2 * nph * Rw
  const int4 *meta;     // per vector {off, n, dx, dy}
  const int32_t *pix;   // [Mc] path pixel offsets, (dx & 0xffff) | (dy << 16)
  uint32_t *rec;        // [W*H][plane A phases, plane B phases][Rw]
  uint8_t *ones;        // [nv][oplane]: per vector, 8 x 8-pixel tiles of 64 bytes (ones_at)
  int64_t oplane;       // bytes per vector: ceil(W/8) * ceil(H/8) * 64
  const int32_t *vbit;  // [Mc] (v << 8) | n of the vector of each record bit
  unsigned mask;        // phases kept (LPF_PHASE0 | LPF_PHASE1 bits)
  // Monte-Carlo position set (packed like the image), nullptr = every placement.  A placement
  // outside it keeps ones + 128 (n <= 126), which meets no plane condition before or after any
  // interchange, so it never counts.
  const uint64_t *sample;
  int end_wgs;          // update workgroups of the step's end (rec_end_workgroups)
  // build scratch: the image (and position set) as periodically extended rows of ew 32-bit
  // words (ew = ceil(W / 32) + 2), and per vector and plane the placement conditions as rows of
  // cw words extended periodically past W (cw = ceil(W / 32) + 2 rounded as (W - 1) / 32 + 3)
  uint32_t *ext, *cond;
  int ew, cw;
  // per vector v with 0 < n < 64, at 2 off(v) - v + t (t = 0 .. 2n): the path indices k whose
  // minor error term (2 k e + n) mod 2n is at least t (e the minor extent), bit k
  const uint64_t *emask;
};

struct AnnealDev;
// Arguments of a step's candidate draws (draw_dev.h).  S_acc, ctl: when given, also zeroed for
// the step (the step's reset folded into the draw).  T_cur (when given) receives the step's
// temperature: T_sched[step - T_base] when T_sched is given, else T.  rank_score (when given):
// the draws' rank keys go to rank_keys and each 256-draw workgroup's best kRankTop to
// rank_lists, for launch_rank_merge.
struct ProposeArgs {
  const AnnealDev *st;
  const uint64_t *bits;
  int W, H;
  uint64_t seed;
  int K, proposal;
  const double *cw1, *cw0;
  double eps;
  int2 *cand;
  double *U;
  int2 *slot;
  int64_t *S_acc;
  StepCtl *ctl;
  const double *T_sched;
  int64_t T_base;
  double T;
  double *T_cur;
  const float *rank_score;
  uint64_t *rank_keys, *rank_lists;
  // uniform draws: the next step's first 64 candidates, drawn during this step (int4 {a, b, tag,
  // 0} at (step & 1) * 64 + k, tag = (step & 0x3fffffff) + 1, pixels as the lists hold them
  // before this step's interchange), so that the next round 0 neither runs the counter-based
  // generator nor reads the lists; null: none
  int4 *pre;
};
struct StepLaunch {
  bool s2;                   // descriptor: two-point probability (k_s2.hip), else lineal path
  const int32_t *s2vec;      // S2: canonical vectors, (dx & 0xffff) | (dy << 16)
  bool records;              // evaluation method: placement-state records, else recount
  bool reset_done;           // ctl and S_acc already zeroed by the candidate draw
  bool ordered;              // candidates are (phase-1 pixel, phase-0 pixel) pairs
  const uint32_t *E;
  DeltaGeo geo;
  const uint64_t *bits;
  uint64_t *bits_rw;
  int W, H;
  const int2 *cand;
  const int2 *slot;
  const double *U;           // nullptr: energies only, no decision
  const int32_t *order;      // evaluation order of the candidates, nullptr: draw order
  int K;                     // candidates per step
  std::vector<RoundPlan> rounds;
  const uint32_t *runs;
  unsigned phase_mask;
  int nv, nterms;            // nterms = phases * vectors
  RecGeo rg;
  const uint32_t *counts;
  uint32_t *counts_rw;
  const uint32_t *target;
  int64_t N, Nt;
  const double *T;           // device: the step's temperature (written by k_propose)
  int64_t out_base;          // >= 0: the step's record goes to out[step - out_base]
  int64_t *S_acc;            // [K] exact energy sums
  int16_t *dl;               // per (term t, candidate k) at t * dl_t + k * dl_k
  int64_t dl_t, dl_k;
  StepCtl *ctl;
  struct AnnealDev *st;
  double *e;
  int32_t *k_sel;
  struct StepResult *out;
  bool use_lds;
  // records method, unranked draws, K > 64: round 0 draws its own candidates in the launch of
  // the draws (draw) and adds its energy sums into S0 (64 entries, zero at the start of a step)
  bool fuse_draw;
  ProposeArgs draw;
  int64_t *S0;
  // records method, ranked draws, K > 64: every round-0 workgroup merges the ranking's workgroup
  // lists (rank_keys + kRankMax) itself, and one writes the order (order_rw) for the later rounds;
  // round 0 adds its sums into S0 and also does the step's resets (ctl, S_acc, the temperature
  // T_cur from T_sched[step - T_base] or T_value), so that its draws may come from the previous
  // step's end
  bool fuse_rank;
  const uint64_t *rank_keys;
  int32_t *order_rw;
  double *T_cur;
  const double *T_sched;
  int64_t T_base;
  double T_value;
  // ranked records chains: the end of this step also draws the next step (next: its arguments in
  // device memory, drawing into the other half of the double-buffered cand / slot / U)
  bool draw_next;
  const ProposeArgs *next;
};

hipError_t launch_ext3(const uint64_t *bits, int W, int H, const DeltaGeo &geo, uint32_t *E,
                       hipStream_t stream);
// Same, skipped on the device when *flag < 0 (no interchange was applied).
hipError_t launch_ext3_if(const uint64_t *bits, int W, int H, const DeltaGeo &geo, uint32_t *E,
                          const int32_t *flag, hipStream_t stream);

// Device-side annealing state (k_anneal.hip).
struct AnnealDev {
  uint64_t step;
  int32_t n1, n0;
  int32_t *pos1, *pos0;  // phase-1 / phase-0 pixel lists (n1 and n0 entries)
  int32_t last_a, last_b;  // the last step's accepted interchange, -1 when none
};
// Same layout as lpf_step_result in include/lpf.h.
struct StepResult {
  int32_t k, a, b, pad;
  double de, e;
  uint64_t step;
};
// End of a step: the decision of the last round (when no earlier round accepted) and the state
// upkeep (control block, counts += dL, image bits, pixel lists, energy, record, step counter).
struct FinalArgs {
  AnnealDev *st;
  StepCtl *ctl;
  const int2 *cand;
  const int2 *slot;
  const int16_t *dl;
  int64_t dl_t, dl_k;
  int nterms;
  int64_t N, Nt;
  double *e_io;
  uint32_t *counts;
  uint64_t *bits;
  int W;
  int32_t *k_sel;
  StepResult *out;
  const int64_t *S_acc;
  const double *U;
  const double *Tp;
  const int32_t *order;
  int li0, lC;         // the last round: evaluation positions li0 .. li0 + lC - 1
  int64_t out_base;    // >= 0: the record goes to out[step - out_base]
  int64_t *S0;         // when given: round 0's sums of a fused round 0, cleared here
};
// Evaluation order of a step's K candidates: the kRankTop draws with the highest predicted gain
// score[a] + score[b] among the first min(K, kRankMax) (best first, ties by draw index, void
// draws lowest), then every other draw in draw order.  Rank scratch: kRankMax keys and
// kRankMax / 256 lists of kRankTop keys (uint64).
constexpr int kRankMax = 4096;
constexpr int kRankTop = 64;
constexpr size_t kRankScratch = sizeof(uint64_t) * (kRankMax + (kRankMax / 256) * kRankTop);
hipError_t launch_propose(const ProposeArgs &p, hipStream_t stream);
// scratch: 4 * ceil(W*H / 1024) doubles
hipError_t launch_learn_weights(const AnnealDev *st, const float *score, double beta, double *cw1,
                                double *cw0, int64_t N, double *scratch, hipStream_t stream);
hipError_t launch_copy_cand(const int2 *cand, int K, int32_t *out, hipStream_t stream);
// Evaluation order from the keys and lists that launch_propose (or launch_rank) wrote.
hipError_t launch_rank_merge(const uint64_t *lists, const uint64_t *keys, int K, int32_t *order,
                             hipStream_t stream);
// Evaluation order of given candidates (keys and lists: the rank scratch).
hipError_t launch_rank(const int2 *cand, const float *score, int K, int32_t *order,
                       uint64_t *keys, uint64_t *lists, hipStream_t stream);
// Exact energy change of K given interchanges on a chain's state: de[i] = S_i / (N^2 Nt).
hipError_t launch_energy(const StepLaunch &L, double *de, hipStream_t stream);
// Placement-state records: build ones and records from the packed image; end a step (its
// decision and upkeep, and the accepted interchange applied to ones and records) in one launch.
hipError_t launch_rec_build(const RecGeo &g, const uint64_t *bits, hipStream_t stream);
hipError_t launch_rec_set_next(ProposeArgs *dst, const ProposeArgs &a0, const ProposeArgs &a1,
                               hipStream_t stream);
// next (ranked chains, device memory): the arguments of the next step's draws, made in the same
// launch by ndraw extra workgroups; nullptr: none.
hipError_t launch_rec_step_end(const RecGeo &g, const FinalArgs &f, const ProposeArgs *next,
                               int ndraw, hipStream_t stream);
// Update workgroups of the records method's step end on a device of `cus` compute units.
int rec_end_workgroups(const RecGeo &g, int cus);
hipError_t launch_rec_round(const StepLaunch &L, const RoundPlan &r, bool decide,
                            hipStream_t stream);
// Round 0 (r.C <= 64 candidates) together with the step's draws L.draw (L.fuse_draw).
hipError_t launch_rec_draw_round0(const StepLaunch &L, const RoundPlan &r, hipStream_t stream);
// Round 0 (r.C = 64 candidates) together with the merge of the ranking (L.fuse_rank).
hipError_t launch_rec_rank_round0(const StepLaunch &L, const RoundPlan &r, hipStream_t stream);
hipError_t launch_init_lists(AnnealDev *st, const uint64_t *bits, int W, int H,
                             hipStream_t stream);
hipError_t launch_lse(const uint32_t *counts, const uint32_t *target, int64_t nterms, int64_t N,
                      int64_t Nt, double *e, hipStream_t stream);
hipError_t launch_delta(const DeltaLaunch &L, hipStream_t stream);
hipError_t prepare_delta_kernels(int max_lds_bytes);
// Offset-row deltas (plan_delta.hip, k_delta.hip).  build_diag_table: false when the table
// would exceed max_bytes.
bool build_diag_table(int cx, int cy, int nchunks, size_t max_bytes, DiagTable &t);
DiagGeo diag_geometry(int W, int H, int cx, int cy);
hipError_t launch_dframe(const uint64_t *bits, int W, int H, const DiagGeo &g, uint32_t *F,
                         hipStream_t stream);
hipError_t launch_delta_diag(const DiagLaunch &L, hipStream_t stream);
hipError_t launch_step(const StepLaunch &L, hipStream_t stream);
hipError_t prepare_step_kernels(int max_lds_bytes);

// ---- swap-proposal CNN (k_cnn.hip) ----
constexpr int kCnnParams = 4961;  // W1 288, b1 16, W2 2304, b2 16, W3 2304, b3 16, W4 16, b4 1
struct CnnSample {
  int32_t img, a, b;
  float y;
};
struct CnnBufs {
  float *prm, *mom, *vel;                        // fp32 parameters and Adam moments
  uint16_t *Wf, *Wt;                             // bf16 [3][9][16][16] forward / transposed
  float *W4bf;                                   // head weights rounded to bf16
  uint16_t *X0, *A1, *A2, *A3, *dZ1, *dZ2, *dZ3;  // channels-last activations and gradients
  float *S, *r;                                  // scores, residuals
  int64_t *dS;                                   // score gradient, 2^-40 fixed point
  float *part1, *part2, *part3, *part_h;         // per-block gradient partials
  float *slices;                                 // [64][kCnnParams] partial sums of the partials
};
hipError_t cnn_forward(const CnnBufs &B, const uint64_t *bits, int W, int H, int batch,
                       float *S, hipStream_t s);
// Scores of one image in one launch (bitwise those of cnn_forward with batch 1).
hipError_t cnn_score(const CnnBufs &B, const uint64_t *bits, int W, int H, float *S,
                     hipStream_t s);
hipError_t cnn_grad(const CnnBufs &B, const uint64_t *bits, int W, int H, int batch,
                    const CnnSample *smp, int n, float *grad, float *loss, hipStream_t s);
hipError_t cnn_pack(const CnnBufs &B, hipStream_t s);
hipError_t cnn_adam(const CnnBufs &B, const float *grad, float lr, float b1, float b2, float eps,
                    float c1, float c2, hipStream_t s);
int cnn_conv_blocks(int64_t npix);

// Kernel launchers (defined in k_full.hip).  All enqueue on `stream` and return the HIP status.
hipError_t launch_pack(const uint8_t *img, int W, int H, uint64_t *bits, hipStream_t stream);
// rows >= H rows of the extended image (row r holds pixel row r mod H); 0 = H.
hipError_t launch_ext(const uint64_t *bits, int W, int H, int we, uint32_t *ext,
                      hipStream_t stream, int rows = 0);
// skip: the enhanced evaluation (waves stop a segment once no start pixel can still count).
hipError_t launch_full(const FullImg &I, const FullShape &sh, unsigned phase_mask, bool skip,
                       hipStream_t stream);
// The same counts without a vector table: the waves take the canonical vectors interleaved.
hipError_t launch_full_canon(const FullImg &I, const FullShape &sh, unsigned phase_mask,
                             hipStream_t stream);
size_t full_lds_bytes(const FullShape &sh, int wpg);
int full_wgs_per_cu(int R, bool skip, int wpg, size_t lds_bytes);
// The caller's buffers of one lpf_batch call (device struct, set before each replay).
struct BatchArgs {
  const uint64_t *pool;
  uint32_t *counts;
};
hipError_t launch_batch(const FullImg *imgs, const BatchArgs *args, const int64_t *counts_off,
                        const int2 *items, int n_items, int *counter, int wpg,
                        unsigned phase_mask, size_t lds_bytes, int cnt_off, int n_wg,
                        hipStream_t stream);
hipError_t launch_batch_args(BatchArgs *args, const uint64_t *pool, uint32_t *counts,
                             hipStream_t stream);
hipError_t launch_ext_batch(const FullImg *imgs, int n_images, int max_we, int max_h,
                            const BatchArgs *args, const int64_t *bits_off, uint32_t *ext,
                            const int64_t *ext_off, hipStream_t stream);
hipError_t prepare_full_kernels(int max_lds_bytes);

// Throughput probes (k_peak.hip): kind 0-3 int32 VALU mixes, 4 LDS reads; nwg workgroups of 256
// threads, sink[nwg * 256].  probe_work = lane-operations (or LDS bytes) of one launch.
hipError_t launch_probe(int kind, int64_t iters, int nwg, uint32_t *sink, hipStream_t stream);
double probe_work(int kind, int64_t iters, int nwg);

// ---- 3-D volumes (k_lpf3.hip) ----
// E: extended rows of the volume (row z*H + y, we >= S*R + (cx >> 5) + 1 dwords), vec: the
// canonical 3-D vectors {dx, dy, dz, canonical index} in launch order; counts[p][nv].
hipError_t launch_lpf3(const uint32_t *E, int W, int H, int D, int we, int R, int S,
                       const int4 *vec, int nv, unsigned phase_mask, uint32_t *counts,
                       hipStream_t stream);
// Slabs of zb start planes staged with their cz-plane halo in LDS, each plane with cy periodic
// halo rows above and below ((H + 2 cy) rows of rst dwords in a plane of ps >= (H + 2 cy) rst
// dwords; (zb + cz) * ps dwords in all), counts accumulated with
// atomics (zeroed here first).  vec in launch order (longest first); woff[j] the first of vector
// j's voxel-table entries (n + 1 rounded up to even); walk: the table (woff[nv - 1] + its
// entries int2), written here first when build is set (it depends on ps and rst only); rpl:
// start rows per lane (2 is used only for R <= 4).
hipError_t launch_lpf3_slab(const uint32_t *E, int W, int H, int D, int we, int R, int S, int rst, int ps,
                            int zb, int cz, int cy, const int4 *vec, const int *woff, int2 *walk,
                            bool build, int rpl, int nv, unsigned phase_mask, uint32_t *counts,
                            hipStream_t stream);
hipError_t prepare_lpf3_kernels(int max_lds_bytes);

// ---- two-point probability (k_s2.hip) ----
// Full evaluation: vector families {dx0, dy, nj} (members dx0 + 32 j, j < nj <= J) sorted by
// dy, in groups of at most 256 (one workgroup each), start rows in blocks of rb; acc holds the
// phase-1 sums [nv] before the output is written.
struct S2Launch {
  const uint32_t *E;        // the packed image (rows of 2 ceil(W / 64) dwords), extended by the kernel
  int W, H, we, swd, swdp, J, rb, nrb, rstB, ngroups, cx, cy, layout;
  const int4 *fams;         // dy-sorted families
  const int4 *groups;       // {first, end, dy of first, dy of last}
  size_t lds_bytes;
  // acc: zero on entry; clear: the other of two accumulators (ncap entries each), which the
  // previous call has finished reading and this call's last launch clears for the next call
  uint32_t *acc, *clear;
  int64_t ncap;
  int64_t nv;
  unsigned phase_mask;
  uint32_t *out;
};
hipError_t launch_s2_full(const S2Launch &L, hipStream_t stream);
hipError_t launch_s2_delta(const uint64_t *bits, int W, int H, const int2 *swaps, int n,
                           const int32_t *vec, int64_t nv, unsigned phase_mask, int32_t *delta,
                           hipStream_t stream);
hipError_t launch_s2_round(const StepLaunch &L, const RoundPlan &r, bool decide,
                           hipStream_t stream);
hipError_t prepare_s2_kernels(int max_lds_bytes);

}  // namespace lpf
