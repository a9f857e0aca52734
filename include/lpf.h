/*
 * liblpf -- the entire lineal path function of periodic two-phase pixel images on AMD MI355X
 * (gfx950), after Havelka, Kucerova & Sykora, "Compression and Reconstruction of Random
 * Microstructures using Accelerated Lineal Path Function" (arXiv:1601.04359).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Image.  W x H pixels, periodic in both directions (Sec. 2.1 periodicity assumption, kept for
 *   the lineal path in Sec. 2.2).  x is the column (0 <= x < W), y the row (0 <= y < H).
 *   Phase index = pixel value: phase 0 and phase 1 (the paper's two phases "b"/"w").
 * Bit-packed image ("bits").  uint64 words, row-major, row stride ceil(W/64) words; pixel (x,y)
 *   is bit (x % 64) of word bits[y * ceil(W/64) + x / 64].  Bits beyond W in the last word of a
 *   row are ignored on input and written as zero by lpf_pack.
 * Segments.  For a vector v = (dx,dy) with n = max(|dx|,|dy|), the segment from (0,0) to v is
 *   digitised into n + 1 pixels p_k (Sec. 2.2, Bresenham): along the major axis p_k moves by k,
 *   and the minor coordinate is sgn(m) * floor((2k|m| + n) / (2n)) (ties rounded away from the
 *   origin).  L_i(v) = #{x : I(x + p_k mod (W,H)) == i for all k} -- the count behind Alg.
 *   "L2_eval"; the probability of Sec. 2.2 is L_i(v) / (W H), left to the caller.
 * Domain.  Cutoff (cx,cy), 0 <= cx <= W-1, 0 <= cy <= H-1.  The canonical half domain D_c lists
 *   [0,cx] x [0,cy] row by row (dy outer, dx inner), then [-cx,-1] x [1,cy] row by row; its size
 *   is (cx+1)(cy+1) + cx*cy, and with cx = W-1, cy = H-1 it is the domain of eq. (segments),
 *   2WH - W - H + 1 vectors.  L(-v) is defined as L(v) (eq. (symmetry)).
 * Phases.  phase_mask bit 0 = phase 0, bit 1 = phase 1 (LPF_PHASE0 | LPF_PHASE1 = LPF_BOTH).
 *   nph = number of bits set.  Output arrays hold the phases in increasing order.
 * Output layouts.  LPF_OUT_HALF: uint32 counts[nph][|D_c|] in canonical order.
 *   LPF_OUT_GRID: uint32 counts[nph][2cy+1][2cx+1], element [p][dy+cy][dx+cx], with both v and
 *   -v filled (eq. (symmetry)).
 * Memory.  Pointers are DEVICE pointers unless marked (host).  The caller owns every buffer; the
 *   library only reads/writes them inside the work it enqueues.  lpf_ctx owns its own scratch
 *   memory and cached tables (vector tables, launch plans, graphs).
 * Streams.  Every compute call validates its arguments on the host, enqueues its kernels on
 *   `stream` (a hipStream_t passed as void*; NULL = the default stream) and returns without
 *   synchronising.  Results are valid once the stream has reached that point.  Scratch memory
 *   is per context: use one context per stream (calls on one context must not overlap).
 * Errors.  Arguments are checked before anything is enqueued; on a check failure nothing is
 *   written, LPF_E_INVAL is returned and lpf_last_error() names the argument.  A failing HIP
 *   call returns LPF_E_DEVICE (an asynchronous kernel fault may surface on a later call or on
 *   stream synchronisation).  No C++ exception crosses this interface.
 */
#ifndef LPF_H
#define LPF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lpf_ctx_s *lpf_ctx;
typedef struct lpf_cnn_s *lpf_cnn; /* swap-proposal network, see lpf_cnn_create */

typedef enum {
  LPF_OK = 0,
  LPF_E_INVAL = -22,
  LPF_E_NOMEM = -12,
  LPF_E_DEVICE = -5,
  LPF_E_UNSUPPORTED = -95
} lpf_status;

enum { LPF_PHASE0 = 1u, LPF_PHASE1 = 2u, LPF_BOTH = 3u };
enum { LPF_OUT_HALF = 0, LPF_OUT_GRID = 1 };

/* Create a context bound to HIP device `hip_device` (made current for the context's own
 * allocations).  *out (host) receives the handle.  Errors: LPF_E_INVAL for a bad device or NULL
 * out, LPF_E_NOMEM when host memory runs out. */
lpf_status lpf_ctx_create(int hip_device, lpf_ctx *out);

/* Release the context's scratch memory and caches.  Waits for the device first.  NULL is a
 * no-op. */
void lpf_ctx_destroy(lpf_ctx ctx);

/* Message of the last failing call on this host thread; never NULL ("" when none). */
const char *lpf_last_error(void);

/* |D_c| = (cx+1)(cy+1) + cx*cy for cx, cy >= 0 (eq. (segments) with a cutoff); -1 when negative. */
int64_t lpf_num_vectors(int cx, int cy);

/* Write the canonical half domain as int16 pairs dxdy[2i] = dx, dxdy[2i+1] = dy (host buffer of
 * 2*|D_c| int16).  Errors: LPF_E_INVAL for negative or > 32767 cutoffs or NULL dxdy. */
lpf_status lpf_vectors(int cx, int cy, int16_t *dxdy);

/* Pack a uint8 image (row-major W*H bytes, nonzero = phase 1) into the bit layout above: the
 * phase image that Alg. "L2_eval" reads pixel by pixel (its input A, whose 2 x 2 periodic tiling
 * the paper builds on the host, Sec. 3.1) held as 64 pixels per word; the periodic halo is added
 * on the device by each evaluation, so no tiled copy is made.
 * bits: ceil(W/64) * H uint64, written in full (padding bits zero).  One kernel launch.
 * Errors: LPF_E_INVAL for NULL pointers or W, H outside [1, 65535]. */
lpf_status lpf_pack(lpf_ctx ctx, const uint8_t *img, int W, int H, uint64_t *bits, void *stream);

/* Entire lineal path function of one image (Sec. 2.2 definition; Alg. "L2_eval" result) for every
 * vector of D_c and every phase of phase_mask, exact uint32 counts in `out_layout`.
 * bits: packed image as above (read only).  counts: see "Output layouts" (written in full).
 * Requires 1 <= W, H <= 65535, 0 <= cx <= W-1, 0 <= cy <= H-1, phase_mask in {1,2,3}.
 * Rows are staged in LDS with their periodic halo; when a row tile and its cy halo rows do not
 * fit (e.g. the whole domain, cx = W - 1, cy = H - 1, of a 1024 x 1024 image), the rows are read
 * from a periodically extended copy of the image in device memory instead (same counts).
 * Errors: LPF_E_INVAL (arguments), LPF_E_UNSUPPORTED (a cutoff above 32767, the int16 range of
 * the vectors, or W > 32768), LPF_E_NOMEM / LPF_E_DEVICE (HIP).  The same cutoff limit applies to
 * every entry point below. */
lpf_status lpf_full(lpf_ctx ctx, const uint64_t *bits, int W, int H, int cx, int cy,
                    unsigned phase_mask, int out_layout, uint32_t *counts, void *stream);

/* The paper's "enhanced" evaluation (Sec. 3.2: segments whose shorter overlapping segments
 * already have no occurrence are not walked to the end), done exactly per wavefront: every 16
 * segment pixels a wavefront stops walking the segment once none of its start pixels can still
 * count for a requested phase.  Same arguments, same counts as lpf_full, bit for bit; the time
 * saved depends on the image.  Errors as lpf_full. */
lpf_status lpf_full_enhanced(lpf_ctx ctx, const uint64_t *bits, int W, int H, int cx, int cy,
                             unsigned phase_mask, int out_layout, uint32_t *counts,
                             void *stream);

/* The Monte-Carlo approximation the paper compares with (Sec. 3, opening paragraph; Sec. 5
 * reconstruction study): segments are compared with the image only at a chosen set X of start
 * positions, counts[p][i] = #{x in X : every pixel of x + path(v_i) is in phase p} (divide by
 * |X| for the approximated probability).  sample: packed mask of X (device, same layout as bits,
 * bit set = start pixel in X; bits past W ignored), read only.  With every bit set this is
 * lpf_full.  Other arguments and errors as lpf_full (LPF_E_INVAL also for sample == NULL). */
lpf_status lpf_full_sampled(lpf_ctx ctx, const uint64_t *bits, int W, int H, int cx, int cy,
                            unsigned phase_mask, int out_layout, const uint64_t *sample,
                            uint32_t *counts, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): the counts of lpf_full, bit for bit, from a call that
 * allocates nothing.  Its only scratch, the periodically extended image (H rows of
 * ceil(W/32) rounded up to the lane layout, plus cx/32 + 1 dwords), lives in a fixed 4 MiB
 * device array of the library (one per GPU, held until the process ends); it uses no vector
 * table (each wavefront derives its vectors from their canonical indices), so nothing is cached
 * either.  Every call on one GPU shares that array: calls that overlap on one GPU (any context,
 * any stream) race and must be serialised by the caller.  Arguments, layouts and errors as
 * lpf_full, plus LPF_E_UNSUPPORTED when the extended image exceeds 4 MiB (W = H = 4096 with
 * cx = 128 needs 4096 * 133 * 4 bytes = 2.1 MiB and fits; W = H = 8192 does not) or when a row
 * tile and its halo rows do not fit in LDS (lpf_full then reads rows from device memory). */
lpf_status lpf_full_noalloc(lpf_ctx ctx, const uint64_t *bits, int W, int H, int cx, int cy,
                            unsigned phase_mask, int out_layout, uint32_t *counts, void *stream);

/* Statistics of the chains lpf_full walks for cutoff (cx, cy) (host only; no device, no
 * context).  A chain is one walked vector v and every vector u of D_c whose digitised path is,
 * up to a translation, pixels 0..n_u of v's path (a "shorter overlapping segment" of v, Sec.
 * 3.2); one walk gives the counts of all of them.  out (host, 4 int64): |D_c|, number of chains,
 * pixels walked per 32 start pixels (sum over chains of the walked length + 1), and M_c = sum
 * over D_c of (n + 1), the pixels a walk per vector would take.  Returns LPF_E_INVAL for a NULL
 * out or a cutoff outside [0, 32767], LPF_E_UNSUPPORTED above 2^26 vectors; sets no message. */
lpf_status lpf_chain_stats(int cx, int cy, int64_t *out);

/* Host check of the launch plan lpf_full builds for cutoff (cx, cy) with nb_want workgroup bins
 * requested (host only; no device, no context): every vector of D_c is counted exactly once,
 * each as pixel l of a walked path whose first l + 1 pixels are its own path (checked by the
 * digitisation rule), members of a piece in increasing l, at most 256 members per bin.  out
 * (host, 4 int64): bins, chain pieces, largest members in a bin, pixels walked.  Returns LPF_OK
 * when every check holds, LPF_E_INVAL when one fails or for a NULL out, a cutoff outside
 * [0, 4096] or nb_want < 1; sets no message. */
lpf_status lpf_plan_check(int cx, int cy, int64_t nb_want, int64_t *out);

/* Throughput probe (diagnostic; not part of the method): one launch of nwg workgroups of 256
 * threads whose lanes each run 8 independent dependency chains for `iters` iterations of
 *   kind 0: two funnel shifts (v_alignbit_b32), a 3-input AND (v_bitop3_b32) and a 3-input OR
 *           (v_or3_b32) -- the instruction mix of the path product in lpf_full;
 *   kind 1: 3-input bitwise ops only;  kind 2: funnel shifts only;  kind 3: popcounts;
 *   kind 4: LDS reads of 16 bytes per lane, conflict-free, 8 per iteration.
 * *work (host, may be NULL) receives the launch's int32 lane-operations (kinds 0-3) or LDS bytes
 * read (kind 4); divided by the launch's time on `stream` this is the sustained rate that
 * roofline fractions are quoted against.  sink: uint32[nwg * 256] (device), written with
 * values of no meaning.  Errors: LPF_E_INVAL (kind outside 0..4, iters outside [1, 2^40], nwg
 * outside [1, 65536], NULL), LPF_E_DEVICE. */
lpf_status lpf_peak_probe(lpf_ctx ctx, int kind, int64_t iters, int nwg, uint32_t *sink,
                          double *work, void *stream);

/* Exact change of the lineal path function under pixel interchanges (Sec. 4 modification
 * operator: the values of pixels a and b are exchanged, which preserves the volume fractions).
 * swaps: int32[n][2] linear pixel indices y*W + x (device).  delta: int32[n][nph][|D_c|] (device,
 * written in full) with delta[s][p][i] = L_p(I')(v_i) - L_p(I)(v_i), canonical vector order.
 * An interchange of two pixels of the same phase, a == b, or an index outside [0, W*H) gives an
 * all-zero row (indices live on the device and are not checked on the host).  Only the
 * translations whose segment covers a or b are recounted: by offset rows (for cutoffs up to 255,
 * a per-cutoff table of at most 256 MB built on the first call) or by runs of start columns
 * (any cutoff; see lpf_set_delta_method).  Same requirements on W, H, cx, cy, phase_mask as
 * lpf_full; 0 <= n <= 2^24.  Errors: LPF_E_INVAL, LPF_E_NOMEM, LPF_E_DEVICE. */
lpf_status lpf_delta_swap(lpf_ctx ctx, const uint64_t *bits, int W, int H, int cx, int cy,
                          unsigned phase_mask, const int32_t *swaps, int n, int32_t *delta,
                          void *stream);

/* How later lpf_delta_swap calls on ctx recount (the results are identical):
 * LPF_SWAP_AUTO: offset rows -- for a fixed difference d between a path index and a placement
 *   index, the pixels of all placements of a vector lie on one image row (column) at two
 *   neighbouring offsets, so one 32-bit window gives the pixel word of up to 32 placements --
 *   when the cutoff's table fits, else runs;
 * LPF_SWAP_RUNS: runs of contiguous start columns, one path product per start row.
 * Errors: LPF_E_INVAL (NULL ctx, other method). */
enum { LPF_SWAP_AUTO = 0, LPF_SWAP_RUNS = 1 };
lpf_status lpf_set_delta_method(lpf_ctx ctx, int method);

/* ---- 3-D volumes (the extension of Sec. 2; the ensemble of cuts of Sec. 6.3) ---------------- */

/* Canonical half of the 3-D cutoff box: the 2-D half domain (lpf_vectors order) at dz = 0, then
 * for dz = 1..cz the rectangle [-cx,cx] x [-cy,cy] row by row (dy outer).  Count
 * |D_c|(cx, cy) + cz (2cx+1)(2cy+1), or -1 for a negative cutoff. */
int64_t lpf_num_vectors3(int cx, int cy, int cz);
/* dxdydz: int16[n][3] (host).  Errors: LPF_E_INVAL (cutoff outside [0, 32767], NULL). */
lpf_status lpf_vectors3(int cx, int cy, int cz, int16_t *dxdydz);

/* Entire lineal path function of a periodic W x H x D two-phase volume: counts[p][i] (uint32,
 * device, written in full) = number of voxels x with every voxel of x + path(v_i) in phase p,
 * for the canonical 3-D vectors and the phases of phase_mask.  The digitised 3-D segment: n =
 * max(|dx|,|dy|,|dz|), major axis the first of x, y, z with extent n, every minor coordinate
 * sgn(m) floor((2k|m| + n)/(2n)) (the 2-D rule per axis).  bits: the volume as D*H packed rows
 * (row z*H + y, lpf_pack of the (D*H) x W byte array), read only.  With cz = 0 the counts are the
 * sums over the D xy-cuts of their 2-D functions (lpf_full), the ensemble average of Sec. 6.3 times
 * D*W*H.  Requires 1 <= W, H, D <= 65535, W*H*D < 2^32, 0 <= cx <= W-1, 0 <= cy <= H-1,
 * 0 <= cz <= D-1, cutoffs <= 32767, phase_mask in {1,2,3}.  The first call for a cutoff and a
 * volume shape allocates the vector list and the segments' voxel table in the context (device
 * memory kept until lpf_destroy; later calls only read them), so a call to be captured in a
 * graph follows one made outside the capture.
 * Errors: LPF_E_INVAL, LPF_E_UNSUPPORTED (W > 32768, too many vectors), LPF_E_NOMEM,
 * LPF_E_DEVICE. */
lpf_status lpf_full3d(lpf_ctx ctx, const uint64_t *bits, int W, int H, int D, int cx, int cy,
                      int cz, unsigned phase_mask, uint32_t *counts, void *stream);

/* ---- two-point probability (Sec. 2.1, eq. (S2dis)), the descriptor compared with in Secs. 5 and 6.1 --- */

/* Two-point counts C_p(v) = W H S2^p(v): the number of pixels x of the periodic image with x and
 * x + v both in phase p, for every vector v of D_c (only its end point matters, no segment) and
 * every phase of phase_mask, exact uint32 counts in `out_layout` (GRID: the entry of -v equals
 * that of v).  The paper evaluates S2 through the FFT over all W x H shifts; here the pairs are
 * counted directly, 32 start pixels per AND and popcount (cx = W-1, cy = H-1 covers every
 * shift).  Phase 0 follows from phase 1 by eq. (S2add) in counts: C_0(v) = W H - 2 N_1 + C_1(v).
 * bits, counts, W, H, cx, cy, phase_mask, out_layout: as lpf_full.
 * Errors: LPF_E_INVAL (arguments), LPF_E_NOMEM / LPF_E_DEVICE (HIP). */
lpf_status lpf_s2(lpf_ctx ctx, const uint64_t *bits, int W, int H, int cx, int cy,
                  unsigned phase_mask, int out_layout, uint32_t *counts, void *stream);

/* Exact change of the two-point counts under pixel interchanges: delta[s][p][i] =
 * C_p(I')(v_i) - C_p(I)(v_i), canonical order, from the closed form over the pairs that contain
 * a or b (the same value for both phases, since N_1 is unchanged).  Arguments, the zero rows and
 * the errors as lpf_delta_swap. */
lpf_status lpf_s2_delta_swap(lpf_ctx ctx, const uint64_t *bits, int W, int H, int cx, int cy,
                             unsigned phase_mask, const int32_t *swaps, int n, int32_t *delta,
                             void *stream);

/* One image of a batch: its size, cutoff, the offset of its packed rows in bits_pool (uint64
 * words) and of its counts in counts_pool (uint32 elements, sized for the batch's layout). */
typedef struct {
  int32_t W, H, cx, cy;
  int64_t bits_off;
  int64_t counts_off;
} lpf_image_desc;

/* lpf_full for many images of any sizes in ONE persistent launch: workgroups draw work items
 * (image, bin of vector chains) from a device counter, longest first, until the list is empty.
 * descs (host): n_images (<= 65535) descriptors; every image follows lpf_full's rules.  The
 * first call for a set of (descriptors, phases, layout) builds launch plans and captures the
 * launch sequence in a hipGraph owned by the context; later calls with the same set replay it,
 * with any bits_pool and counts_pool (their addresses are written on `stream` before each
 * replay).  The context keeps the 16 most recently used graphs (releasing one waits for the
 * device).  Calls on one context must not overlap (the graph's scratch is shared).  Shapes tuned
 * by lpf_autotune_full for an image size are used.  Errors: LPF_E_INVAL (a descriptor, naming
 * its index), LPF_E_UNSUPPORTED, LPF_E_NOMEM, LPF_E_DEVICE. */
lpf_status lpf_batch(lpf_ctx ctx, const uint64_t *bits_pool, const lpf_image_desc *descs,
                     int n_images, unsigned phase_mask, int out_layout, uint32_t *counts_pool,
                     void *stream);

/* Autotuner for lpf_full: times the tile shapes R in {2,4,8,16}, waves per group in {4,8} (and
 * 16 with the 160 KiB budget, one group per CU) and staging budgets {64 KiB, 160 KiB} on the
 * given image (several runs each, stream-ordered and
 * synchronised here) and records the fastest for images of this W, H, cx, cy in the context;
 * lpf_full and lpf_batch then use it.  *best_ms (host, may be NULL) receives its time.  This
 * replaces the paper's fixed occupancy rule, eq. (block).  Errors: as lpf_full. */
lpf_status lpf_autotune_full(lpf_ctx ctx, const uint64_t *bits, int W, int H, int cx, int cy,
                             unsigned phase_mask, void *stream, double *best_ms);

/* The shape recorded by lpf_autotune_full for W, H, cx, cy (host outputs, each may be NULL).
 * Errors: LPF_E_INVAL when none was recorded. */
lpf_status lpf_get_tuned_shape(lpf_ctx ctx, int W, int H, int cx, int cy, int *R,
                               int *waves_per_group, int *lds_bytes);

/* ---- simulated annealing (Sec. 4, Alg. "annealing"; objective eq. (LSE)) ------------------ */

typedef struct lpf_anneal_s *lpf_anneal;

/* One step's record (device).  accepted_k = index of the applied candidate in draw order, or -1
 * when none passed; a = the phase-1 pixel that became phase 0, b = the phase-0 pixel that became
 * phase 1; delta_e = its energy change; e = energy after the step; step = the step's index. */
typedef struct {
  int32_t accepted_k, a, b, reserved;
  double delta_e, e;
  uint64_t step;
} lpf_step_result;

enum { LPF_PROP_UNIFORM = 0, LPF_PROP_INTERFACIAL = 1, LPF_PROP_LEARNED = 2 };

/* Create an annealing chain on a W x H image (the "cell").  The caller owns and keeps alive:
 *   bits    packed image (device), updated in place by every accepted step;
 *   counts  uint32[nph][|D_c|] (device), written here with L(bits) and kept equal to it;
 *   target  uint32[nph][|D_c|] (device, read only): exact counts of the original image over Nt
 *           pixels (Nt >= 1), e.g. from lpf_full on that image with the same cutoff and phases;
 *   e       one double (device), written here with eq. (LSE), sum over the mask's phases and D_c
 *           of (target/Nt - counts/(W*H))^2, and updated by every accepted step.
 * pos: NULL, or int32[W*H] (device) holding the phase-1 pixel list (n1 entries) followed by the
 *   phase-0 list (a chain exported by lpf_anneal_export); NULL builds both lists in ascending
 *   pixel order.  n1 is read only when pos is given.  seed and step0 select the random stream:
 *   candidate k of step s uses Philox-4x64-10 with counter {s, k, 0, 0} and key {seed, 0x6c7066}:
 *   a = pos1[(r0>>32)*n1 >> 32], b = pos0[(r1>>32)*n0 >> 32], U = (r2>>11) * 2^-53.
 * Requires an image with both phases present; same W, H, cx, cy, phase_mask rules as lpf_full,
 * and max(cx, cy) <= 16383.  Energy changes are exact int64 sums: creation fails with
 * LPF_E_UNSUPPORTED when nph * |D_c| * d * Nt * (d + 4 W H), d = 2 (max(cx, cy) + 1), exceeds
 * 2^63 - 1 (e.g. a 256 x 256 cell, cutoff 48, both phases, Nt = 2048^2 gives 1.0e18).
 * Errors: LPF_E_INVAL, LPF_E_NOMEM, LPF_E_DEVICE, LPF_E_UNSUPPORTED. */
lpf_status lpf_anneal_create(lpf_ctx ctx, uint64_t *bits, int W, int H, int cx, int cy,
                             unsigned phase_mask, uint32_t *counts, const uint32_t *target,
                             int64_t Nt, uint64_t seed, uint64_t step0, const int32_t *pos,
                             int n1, double *e, lpf_anneal *out, void *stream);

/* An annealing chain with the two-point probability as the descriptor (the S2-based
 * reconstruction the paper compares with, Sec. 5): counts receives lpf_s2 of the cell (HALF
 * layout) and target holds lpf_s2 counts of the original image over Nt pixels; the energy is
 * eq. (LSE) over those counts.  Every other argument, and every other lpf_anneal_* call, as for
 * lpf_anneal_create; the exact int64 bound uses d = 6 (the largest change of one S2 count).
 * lpf_anneal_set_method accepts only LPF_DELTA_AUTO for such a chain and lpf_anneal_get_method
 * returns LPF_DELTA_S2.  Errors: as lpf_anneal_create. */
lpf_status lpf_anneal_create_s2(lpf_ctx ctx, uint64_t *bits, int W, int H, int cx, int cy,
                                unsigned phase_mask, uint32_t *counts, const uint32_t *target,
                                int64_t Nt, uint64_t seed, uint64_t step0, const int32_t *pos,
                                int n1, double *e, lpf_anneal *out, void *stream);

/* An annealing chain driven by the Monte-Carlo approximation (the paper's reconstruction from
 * the approximated function, Sec. 5): sample is the cell's position set X (device, packed like
 * bits, read only, kept alive by the caller); counts receives lpf_full_sampled of the cell over X
 * and target holds the original's sampled counts over its own Nt positions; the objective is
 * eq. (LSE) with N = |X| (the approximated probabilities counts/|X| and target/Nt).  Every
 * candidate's change is exact for the sampled counts.  Uses the records method (only it carries
 * a position set): requires max(cx, cy) <= 126 and the records' memory; lpf_anneal_set_method
 * refuses LPF_DELTA_RECOUNT.  Other arguments and calls as lpf_anneal_create.
 * Errors: as lpf_anneal_create (LPF_E_INVAL also for a NULL or empty sample). */
lpf_status lpf_anneal_create_sampled(lpf_ctx ctx, uint64_t *bits, int W, int H, int cx, int cy,
                                     unsigned phase_mask, const uint64_t *sample,
                                     uint32_t *counts, const uint32_t *target, int64_t Nt,
                                     uint64_t seed, uint64_t step0, const int32_t *pos, int n1,
                                     double *e, lpf_anneal *out, void *stream);

/* One step: draw n_candidates interchanges (a phase-1 pixel with a phase-0 pixel; with
 * LPF_PROP_INTERFACIAL a draw where either pixel has no 4-neighbour of the other phase is void),
 * compute each one's exact energy change de against the current state, and apply the first, in
 * draw order, with de <= 0 or U < exp(-de/T) (the Metropolis rule for a minimisation).  The
 * candidates are evaluated in rounds (64 candidates, then the rest, at most 8192 per round) and rounds after an acceptance are skipped, which gives the same result as
 * evaluating all of them.  The step's record is written to *out (device).  Everything stays on
 * the device.
 * Errors: LPF_E_INVAL (n_candidates outside [1, 2^20], proposal, T <= 0), LPF_E_NOMEM,
 * LPF_E_DEVICE. */
lpf_status anneal_step(lpf_anneal st, int n_candidates, int proposal, double T,
                       lpf_step_result *out, void *stream);

/* nsteps consecutive steps, step i at temperature T_sched[i] (device, double[nsteps]), records
 * to out[i] (device, lpf_step_result[nsteps]); the same chain, bit for bit, as nsteps calls of
 * anneal_step.  The steps are enqueued as replays of a hipGraph of 32 captured steps (the
 * temperature and the record slot are read on the device from the chain's step counter), the
 * remainder one by one; learned proposals are captured only when their re-scoring interval
 * (refresh) divides 32, else enqueued one by one.
 * Nothing is synchronised.  Errors: as anneal_step (LPF_E_INVAL also for nsteps < 0 or NULL
 * buffers when nsteps > 0); temperatures are not checked on the host (they live on the device). */
lpf_status lpf_anneal_run(lpf_anneal st, int n_candidates, int proposal, const double *T_sched,
                          int nsteps, lpf_step_result *out, void *stream);

/* The evaluation order of a ranked learned step: order[0..K) (int32, device) lists the kRankTop
 * = 64 draws with the highest fp32 key score[a] + score[b] among the first R = min(K, 4096)
 * (best first; ties, including -0 and +0, by draw index; a draw with a < 0 or b < 0, or a NaN
 * key, counts as -inf), then every other draw in draw order.  cand: int32[K][2] (device);
 * score: float per pixel (device); scratch (40 KB) from the context, so calls on one context
 * that are in flight on different streams at once race on it.
 * Errors: LPF_E_INVAL (K outside [1, 2^20], NULL), LPF_E_NOMEM, LPF_E_DEVICE. */
lpf_status lpf_rank(lpf_ctx ctx, const int32_t *cand, const float *score, int K, int32_t *order,
                    void *stream);

/* Learned proposals (LPF_PROP_LEARNED): before each draw the cell is scored, by `net` (an
 * lpf_cnn for this cell size, run on the current cell) or, when net is NULL, by the caller's
 * field scores (device, W*H fp32, read at every learned draw).  With probability eps_uniform a
 * candidate is drawn as LPF_PROP_UNIFORM (random stream word r3); otherwise a is drawn from the
 * phase-1 pixels with probability proportional to exp(clamp(beta * score[a], -60, 60)) and b
 * likewise from the phase-0 pixels (inversion of r0, r1 on fp64 prefix sums in pixel-list
 * order); beta = 0 draws exactly the LPF_PROP_UNIFORM candidates (then the scores serve the
 * ranking below only).  The exact energy change still decides acceptance; no proposal-ratio correction is
 * applied (the chain minimises, it does not sample).  refresh >= 1: the scores and prefix sums
 * are recomputed at the first learned draw and then every `refresh` learned draws (steps or
 * lpf_anneal_propose calls); in between, the pixel-list slots keep the weights of the last
 * scoring (an interchange leaves both slots' old weights in place), which only changes which
 * candidates are proposed, never how they are judged.  rank = 1: the network also ranks the
 * step's candidates: the 64 draws with the highest predicted gain score[a] + score[b] (fp32 sum;
 * ties by draw index; void draws lowest) among the first min(K, 4096) are evaluated first, best
 * first, then every other draw in draw order, and the first of that order to pass the Metropolis
 * test is applied (the record's accepted_k is still the draw index); rank = 0 keeps draw order.
 * Errors: LPF_E_INVAL. */
lpf_status lpf_anneal_set_proposal(lpf_anneal st, lpf_cnn net, const float *scores, float beta,
                                   float eps_uniform, int refresh, int rank);

/* The current step's K candidates as int32 (a, b) pairs into cand (device, [K][2]), without
 * evaluating them or advancing the chain (a = -1 marks a void interfacial draw). */
lpf_status lpf_anneal_propose(lpf_anneal st, int K, int proposal, int32_t *cand, void *stream);

/* Exact energy change de[i] (device, double) of n interchanges swaps (device, int32 [n][2]) on
 * the chain's current state, with the same integer formula as anneal_step (invalid or
 * same-phase pairs give 0).  Used to label training samples for the proposal network. */
lpf_status lpf_anneal_delta_energy(lpf_anneal st, const int32_t *swaps, int n, double *de,
                                   void *stream);

/* How a chain evaluates candidates; every method gives the same exact integer changes.
 *   LPF_DELTA_RECOUNT  recount the placements through the two pixels from the image (no state
 *                      beyond three copies of the image; cost grows with the square of the
 *                      segment length per vector and candidate);
 *   LPF_DELTA_RECORDS  keep, for every pixel q, the state of every placement whose segment
 *                      passes through q (bits [ones == 0], [ones == 1], [ones == n], [ones == n+1]
 *                      of its phase-1 pixel count) plus the counts themselves, so that a
 *                      candidate reads two contiguous records; memory W*H*(4*nph*sum(n_v+1)/32
 *                      + |D_c|) bytes, requires max(cx, cy) <= 254;
 *   LPF_DELTA_AUTO     (default) records when they fit in 16 GiB and in half the free device
 *                      memory, else recount.
 * Errors: LPF_E_INVAL, LPF_E_UNSUPPORTED (records for a cutoff above 254 or a too large cell). */
enum { LPF_DELTA_AUTO = 0, LPF_DELTA_RECOUNT = 1, LPF_DELTA_RECORDS = 2, LPF_DELTA_S2 = 3 };
lpf_status lpf_anneal_set_method(lpf_anneal st, int method);

/* The method the chain's next step uses (LPF_DELTA_RECOUNT or LPF_DELTA_RECORDS; LPF_DELTA_S2
 * for a chain made by lpf_anneal_create_s2), -1 on error. */
int lpf_anneal_get_method(lpf_anneal st);

/* Copy the chain's pixel lists to pos (device, int32[W*H]: phase-1 list then phase-0 list) and
 * return, after synchronising the stream, the number of phase-1 pixels and the next step index
 * (host).  With the caller's bits, counts and e this is everything a resumed chain needs. */
lpf_status lpf_anneal_export(lpf_anneal st, int32_t *pos, int *n1, uint64_t *next_step,
                             void *stream);

/* Release the chain's device state (waits for the device).  NULL is a no-op. */
void lpf_anneal_destroy(lpf_anneal st);

/* ---- swap-proposal CNN --------------------------------------------------------------------
 * Not in the paper, which leaves the modification operator open (Sec. 4): a small CNN scores
 * every pixel of a cell so that candidate interchanges can be drawn where they are likely to
 * lower the error; the exact lineal-path change still judges every move (anneal_step).
 * Network: input (pixel value, interface flag) -> 3 x [conv3x3, 16 channels, periodic padding,
 * relu] -> 1x1 head, one score per pixel.  bfloat16 weights and activations, fp32 accumulation
 * (MFMA).  Parameters: LPF_CNN_PARAMS fp32 values packed as W1 [9][16][2], b1 [16],
 * W2 [9][16][16], b2, W3 [9][16][16], b3, W4 [16], b4 [1]; tap t = 3 dy + dx reads the input at
 * offset (dy-1, dx-1).  Training loss for samples (image, a, b, y): mean (S[a] + S[b] - y)^2. */
#define LPF_CNN_PARAMS 4961

typedef struct {
  int32_t img;  /* index of the image in the batch */
  int32_t a, b; /* linear pixel indices y*W + x */
  float y;      /* regression target for S[a] + S[b] */
} lpf_cnn_sample;

/* Network for W x H cells, batches of up to max_batch images and max_samples samples.
 * params: LPF_CNN_PARAMS fp32 values (device), or NULL for all zeros.  Errors: LPF_E_INVAL,
 * LPF_E_NOMEM, LPF_E_DEVICE. */
lpf_status lpf_cnn_create(lpf_ctx ctx, int W, int H, int max_batch, int max_samples,
                          const float *params, lpf_cnn *out, void *stream);
/* Replace the parameters (device, LPF_CNN_PARAMS fp32) and clear the Adam moments. */
lpf_status lpf_cnn_set_params(lpf_cnn net, const float *params, void *stream);
/* Copy the parameters to params (device, LPF_CNN_PARAMS fp32). */
lpf_status lpf_cnn_get_params(lpf_cnn net, float *params, void *stream);
/* Scores of a batch of packed cells (bits: batch images back to back, device) into
 * scores[batch][H][W] (fp32, device).  A single image is scored in one launch (16 x 16 tiles with
 * their halo in LDS), with the same scores bit for bit as the layer-by-layer batch path. */
lpf_status lpf_cnn_forward(lpf_cnn net, const uint64_t *bits, int batch, float *scores,
                           void *stream);
/* Loss and its gradient for n samples on a batch of cells: grad (device, LPF_CNN_PARAMS fp32),
 * loss (device, one fp32).  A sample with an out-of-range image or pixel contributes a zero
 * residual.  The score gradient is accumulated in 2^-40 fixed point, so the result does not
 * depend on the order of the samples.  Errors: LPF_E_INVAL (batch, n), LPF_E_DEVICE. */
lpf_status lpf_cnn_grad(lpf_cnn net, const uint64_t *bits, int batch,
                        const lpf_cnn_sample *samples, int n, float *grad, float *loss,
                        void *stream);
/* One Adam step (Kingma & Ba) with gradient grad (device) at step t >= 1. */
lpf_status lpf_cnn_adam(lpf_cnn net, const float *grad, int t, float lr, float beta1, float beta2,
                        float eps, void *stream);
void lpf_cnn_destroy(lpf_cnn net);

/* Tile-shape override for lpf_full (and the kernels that share its launch plans); used by the
 * autotuner.  R = 32-pixel words per lane (1,2,4,8,16), S = lanes per image row (power of two,
 * <= 64), waves_per_group (1..16; automatic: 8, or 16 when the rows need the 160 KiB budget),
 * lds_bytes = staging budget per workgroup (<= 160 KiB; a
 * budget too small for one row tile and its halo selects rows read from device memory).
 * 0 in any field restores the automatic choice for that field.  This replaces the paper's
 * occupancy rule for the block size, eq. (block).  Errors: LPF_E_INVAL for values out of range.
 * A shape that cannot cover an image makes the later compute call fail with LPF_E_UNSUPPORTED. */
lpf_status lpf_set_full_shape(lpf_ctx ctx, int R, int S, int waves_per_group, int lds_bytes);

#ifdef __cplusplus
}
#endif

#endif /* LPF_H */
