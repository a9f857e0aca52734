/*
 * CPU ORACLE for the entire lineal path function (LPF) -- TEST INFRASTRUCTURE ONLY.
 *
 * Only tests/, the smoke() entry point and the benchmark's cpu_baseline leg may load this
 * file's library.  The product library never links, loads or calls it, and this file includes
 * nothing from the product (no shared headers, tables or helpers).
 *
 * Every routine is the plain definition from Havelka, Kucerova & Sykora, "Compression and
 * Reconstruction of Random Microstructures using Accelerated Lineal Path Function"
 * (arXiv:1601.04359), written out with no blocking, bit-packing or reordering:
 *
 *   - oracle_bresenham      Sec. 2.2 (digitised segments, Bresenham 1965); tie rule below.
 *   - oracle_vectors        Sec. 2.2, eq. (segments) and eq. (symmetry): canonical half domain.
 *   - oracle_lpf*           Sec. 3, Alg. "L2_eval" loop structure (segment x translation x
 *                           pixel with early break) on a periodic image.
 *   - oracle_delta_swap*    Sec. 4 modification operator (two-pixel interchange), evaluated as
 *                           L(I') - L(I): by two full evaluations, and by a recount restricted
 *                           to the translations whose segment covers a swapped pixel.
 *   - oracle_lpf_sampled    Sec. 3 opening: the Monte-Carlo approximation, segments compared at a
 *                           given set of start positions only (and its interchange update and
 *                           chain: oracle_delta_swap_sampled, oracle_anneal_run_sampled).
 *   - oracle_*3             the 3-D extension (Sec. 2): segments, half domain and counts on a
 *                           periodic volume.
 *   - oracle_s2*            Sec. 2.1, eq. (S2dis): two-point probability counts (definition sum).
 *   - oracle_s2_delta_swap  Sec. 4 interchange applied to eq. (S2dis), recounting the pairs that
 *                           contain a swapped pixel.
 *   - oracle_anneal_run     Sec. 4, Alg. "annealing" + eq. (LSE): Metropolis rule on pixel
 *                           interchanges, with the batched first-accept step described there;
 *                           oracle_anneal_run_desc also anneals against S2 (the comparison of Secs. 5 and 6.1);
 *                           oracle_anneal_run_ranked evaluates each step's draws in the ranked
 *                           order of a given score field (reading R18).
 *   - oracle_philox4x64     Salmon et al., SC'11 "Parallel random numbers: as easy as 1, 2, 3",
 *                           Philox-4x64 with 10 rounds.
 *
 * Readings of the paper taken here (each also listed in the design notes):
 *   R1 Bresenham tie rule: minor coordinate = sgn(m) * floor((2k|m| + n) / (2n)), i.e. round half
 *      up in magnitude from the segment origin; implemented incrementally with the error term
 *      initialised to n.  The paper calls the digitisation unique but does not state a rule.
 *      PARITY UNPINNED on tie vectors (n / gcd(n,|m|) even): a convention.
 *   R2 L(-v) is defined as L(v) from the path of the canonical representative v.
 *   R4 a segment of major length n has n + 1 pixels (both ends).
 *   R5 x = column (image width W), y = row (image height H); pixel (x,y) is img[y*W + x].
 *   R8 Metropolis for a minimisation: accept iff de <= 0 or U < exp(-de / T).
 *   R11 phase index = pixel value (0 or 1).
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (see oracle/build.sh).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------------------------
 * Segment digitisation (Sec. 2.2, Bresenham): pixels p_0 = (0,0) ... p_n = (dx,dy), n = max(|dx|,|dy|).
 * Incremental error form of reading R1: err starts at n, grows by 2|m| per major step, and a
 * minor step is taken (err -= 2n) whenever err >= 2n.
 * Returns the pixel count n + 1.
 * ------------------------------------------------------------------------------------------ */
int oracle_bresenham(int dx, int dy, int *px, int *py) {
  int adx = dx < 0 ? -dx : dx, ady = dy < 0 ? -dy : dy;
  int sx = dx < 0 ? -1 : 1, sy = dy < 0 ? -1 : 1;
  int n = adx > ady ? adx : ady;
  if (n == 0) {
    px[0] = 0;
    py[0] = 0;
    return 1;
  }
  int xmajor = adx >= ady;
  int m = xmajor ? ady : adx;
  long err = n;
  int q = 0;
  for (int k = 0; k <= n; ++k) {
    if (k > 0) {
      err += 2L * m;
      if (err >= 2L * n) {
        err -= 2L * n;
        q += 1;
      }
    }
    if (xmajor) {
      px[k] = sx * k;
      py[k] = sy * q;
    } else {
      px[k] = sx * q;
      py[k] = sy * k;
    }
  }
  return n + 1;
}

/* ------------------------------------------------------------------------------------------
 * Segment domain with a cutoff (eq. (segments) with the rectangles clipped to |dx|<=cx, |dy|<=cy;
 * cx = W-1, cy = H-1 gives the paper's domain).  Canonical order: first rectangle
 * [0,cx] x [0,cy] row by row (dy outer, dx inner), then [-cx,-1] x [1,cy] row by row.
 * The other half of the orientations follows from eq. (symmetry).
 * ------------------------------------------------------------------------------------------ */
int64_t oracle_num_vectors(int cx, int cy) {
  return (int64_t)(cx + 1) * (cy + 1) + (int64_t)cx * cy;
}

int oracle_vectors(int cx, int cy, int16_t *dxdy) {
  if (cx < 0 || cy < 0) return -22;
  int64_t i = 0;
  for (int dy = 0; dy <= cy; ++dy)
    for (int dx = 0; dx <= cx; ++dx) {
      dxdy[2 * i] = (int16_t)dx;
      dxdy[2 * i + 1] = (int16_t)dy;
      ++i;
    }
  for (int dy = 1; dy <= cy; ++dy)
    for (int dx = -cx; dx <= -1; ++dx) {
      dxdy[2 * i] = (int16_t)dx;
      dxdy[2 * i + 1] = (int16_t)dy;
      ++i;
    }
  return 0;
}

static inline int wrap(int v, int n) {
  v %= n;
  return v < 0 ? v + n : v;
}

/* ------------------------------------------------------------------------------------------
 * One segment, one phase: Alg. "L2_eval" inner two loops.  For every translation (x,y) of the
 * periodic W x H image, walk the segment's pixels and break at the first pixel that is not in
 * the phase; count the translations that reach the end.
 * ------------------------------------------------------------------------------------------ */
static uint32_t lpf_one(const uint8_t *img, int W, int H, const int *px, const int *py, int np,
                        uint8_t phase) {
  uint32_t count = 0;
  for (int y = 0; y < H; ++y) {
    for (int x = 0; x < W; ++x) {
      int pix;
      for (pix = 0; pix < np; ++pix) {
        int xx = wrap(x + px[pix], W), yy = wrap(y + py[pix], H);
        if (img[(size_t)yy * W + xx] != phase) break;
      }
      if (pix == np) count += 1;
    }
  }
  return count;
}

/* L for an explicit list of vectors (each digitised by oracle_bresenham), for the phases in
 * phase_mask (bit0 = phase 0, bit1 = phase 1); counts[p][i], phase 0 first. */
int oracle_lpf_vectors(const uint8_t *img, int W, int H, const int16_t *dxdy, int64_t nv,
                       unsigned phase_mask, uint32_t *counts, int nthreads) {
  if (W < 1 || H < 1 || nv < 0 || (phase_mask & ~3u) || !phase_mask) return -22;
  int nph = (phase_mask & 1) + ((phase_mask >> 1) & 1);
  int maxlen = (W > H ? W : H) * 2 + 2;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
  int bad = 0;
#pragma omp parallel
  {
    int *px = (int *)malloc(sizeof(int) * maxlen);
    int *py = (int *)malloc(sizeof(int) * maxlen);
#pragma omp for schedule(dynamic, 1)
    for (int64_t i = 0; i < nv; ++i) {
      int dx = dxdy[2 * i], dy = dxdy[2 * i + 1];
      int adx = dx < 0 ? -dx : dx, ady = dy < 0 ? -dy : dy;
      if (adx >= maxlen - 1 || ady >= maxlen - 1) {
#pragma omp atomic write
        bad = 1;
        continue;
      }
      int np = oracle_bresenham(dx, dy, px, py);
      int p = 0;
      for (int ph = 0; ph < 2; ++ph) {
        if (!(phase_mask & (1u << ph))) continue;
        counts[(size_t)p * nv + i] = lpf_one(img, W, H, px, py, np, (uint8_t)ph);
        ++p;
      }
    }
    free(px);
    free(py);
  }
  (void)nph;
  return bad ? -22 : 0;
}

/* Full LPF over the canonical half domain (out_layout 0: counts[nph][|D_c|]) or the full
 * (2cy+1) x (2cx+1) grid (out_layout 1: counts[nph][dy+cy][dx+cx]) where the second half is
 * filled by eq. (symmetry). */
int oracle_lpf(const uint8_t *img, int W, int H, int cx, int cy, unsigned phase_mask,
               int out_layout, uint32_t *counts, int nthreads) {
  if (W < 1 || H < 1 || cx < 0 || cy < 0 || cx > W - 1 || cy > H - 1) return -22;
  if (out_layout != 0 && out_layout != 1) return -22;
  int64_t nv = oracle_num_vectors(cx, cy);
  int16_t *v = (int16_t *)malloc(sizeof(int16_t) * 2 * nv);
  oracle_vectors(cx, cy, v);
  int nph = (phase_mask & 1) + ((phase_mask >> 1) & 1);
  int rc;
  if (out_layout == 0) {
    rc = oracle_lpf_vectors(img, W, H, v, nv, phase_mask, counts, nthreads);
  } else {
    uint32_t *half = (uint32_t *)malloc(sizeof(uint32_t) * nph * nv);
    rc = oracle_lpf_vectors(img, W, H, v, nv, phase_mask, half, nthreads);
    int gw = 2 * cx + 1, gh = 2 * cy + 1;
    for (int p = 0; p < nph; ++p)
      for (int64_t i = 0; i < nv; ++i) {
        int dx = v[2 * i], dy = v[2 * i + 1];
        uint32_t c = half[(size_t)p * nv + i];
        counts[(size_t)p * gw * gh + (size_t)(dy + cy) * gw + (dx + cx)] = c;
        counts[(size_t)p * gw * gh + (size_t)(-dy + cy) * gw + (-dx + cx)] = c;
      }
    free(half);
  }
  free(v);
  return rc;
}

/* ------------------------------------------------------------------------------------------
 * Monte-Carlo approximation (Sec. 3, opening paragraph): the segments are compared with the
 * image only at a chosen set X of start positions.  counts[p][i] = #{x in X : every pixel of
 * x + path(v_i) is in phase p}, canonical half domain; X is given as a W x H byte mask (nonzero
 * = x in X).  With X = every pixel this is oracle_lpf.
 * ------------------------------------------------------------------------------------------ */
int oracle_lpf_sampled(const uint8_t *img, int W, int H, int cx, int cy, unsigned phase_mask,
                       const uint8_t *sample, uint32_t *counts, int nthreads) {
  if (W < 1 || H < 1 || cx < 0 || cy < 0 || cx > W - 1 || cy > H - 1) return -22;
  if (!phase_mask || (phase_mask & ~3u)) return -22;
  int64_t nv = oracle_num_vectors(cx, cy);
  int16_t *v = (int16_t *)malloc(sizeof(int16_t) * 2 * nv);
  oracle_vectors(cx, cy, v);
  int maxlen = (cx > cy ? cx : cy) + 1;
  /* the position set as a list, row by row */
  int64_t ns = 0;
  for (int64_t q = 0; q < (int64_t)W * H; ++q) ns += sample[q] != 0;
  int32_t *pos = (int32_t *)malloc(sizeof(int32_t) * (ns ? ns : 1));
  ns = 0;
  for (int64_t q = 0; q < (int64_t)W * H; ++q)
    if (sample[q]) pos[ns++] = (int32_t)q;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel
  {
    int *px = (int *)malloc(sizeof(int) * maxlen);
    int *py = (int *)malloc(sizeof(int) * maxlen);
#pragma omp for schedule(dynamic, 4)
    for (int64_t i = 0; i < nv; ++i) {
      int np = oracle_bresenham(v[2 * i], v[2 * i + 1], px, py);
      int p = 0;
      for (int ph = 0; ph < 2; ++ph) {
        if (!(phase_mask & (1u << ph))) continue;
        uint32_t count = 0;
        for (int64_t t = 0; t < ns; ++t) {
          const int y = pos[t] / W, x = pos[t] % W;
          int k;
          for (k = 0; k < np; ++k)
            if (img[(size_t)wrap(y + py[k], H) * W + wrap(x + px[k], W)] != ph) break;
          if (k == np) count += 1;
        }
        counts[(size_t)p * nv + i] = count;
        ++p;
      }
    }
    free(px);
    free(py);
  }
  free(pos);
  free(v);
  return 0;
}

/* ------------------------------------------------------------------------------------------
 * Two-point probability (Sec. 2.1, eq. (S2dis)) as integer counts C_p(v) = W H S2^p(v):
 * the number of pixels x of the periodic image with x and x + v both in phase p.  Written as
 * the definition's double sum; the paper evaluates the same sum through the FFT, which the
 * tests use as a pin.  S2 does not depend on any digitised path, only on the end point v.
 * ------------------------------------------------------------------------------------------ */
static uint32_t s2_one(const uint8_t *img, int W, int H, int dx, int dy, uint8_t phase) {
  uint32_t count = 0;
  for (int y1 = 0; y1 < H; ++y1)
    for (int x1 = 0; x1 < W; ++x1)
      if (img[(size_t)y1 * W + x1] == phase &&
          img[(size_t)wrap(y1 + dy, H) * W + wrap(x1 + dx, W)] == phase)
        count += 1;
  return count;
}

/* S2 counts for an explicit list of vectors; counts[p][i], phase 0 first. */
int oracle_s2_vectors(const uint8_t *img, int W, int H, const int16_t *dxdy, int64_t nv,
                      unsigned phase_mask, uint32_t *counts, int nthreads) {
  if (W < 1 || H < 1 || nv < 0 || (phase_mask & ~3u) || !phase_mask) return -22;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t i = 0; i < nv; ++i) {
    int p = 0;
    for (int ph = 0; ph < 2; ++ph) {
      if (!(phase_mask & (1u << ph))) continue;
      counts[(size_t)p * nv + i] = s2_one(img, W, H, dxdy[2 * i], dxdy[2 * i + 1], (uint8_t)ph);
      ++p;
    }
  }
  return 0;
}

/* S2 counts over the canonical half domain (out_layout 0: counts[nph][|D_c|]) or over the whole
 * (2cy+1) x (2cx+1) grid of vectors (out_layout 1: counts[nph][dy+cy][dx+cx]), every grid entry
 * evaluated from the definition (no symmetry is used here). */
int oracle_s2(const uint8_t *img, int W, int H, int cx, int cy, unsigned phase_mask,
              int out_layout, uint32_t *counts, int nthreads) {
  if (W < 1 || H < 1 || cx < 0 || cy < 0 || cx > W - 1 || cy > H - 1) return -22;
  if (out_layout != 0 && out_layout != 1) return -22;
  int64_t nv;
  int16_t *v;
  if (out_layout == 0) {
    nv = oracle_num_vectors(cx, cy);
    v = (int16_t *)malloc(sizeof(int16_t) * 2 * nv);
    oracle_vectors(cx, cy, v);
  } else {
    nv = (int64_t)(2 * cx + 1) * (2 * cy + 1);
    v = (int16_t *)malloc(sizeof(int16_t) * 2 * nv);
    int64_t i = 0;
    for (int dy = -cy; dy <= cy; ++dy)
      for (int dx = -cx; dx <= cx; ++dx, ++i) {
        v[2 * i] = (int16_t)dx;
        v[2 * i + 1] = (int16_t)dy;
      }
  }
  int rc = oracle_s2_vectors(img, W, H, v, nv, phase_mask, counts, nthreads);
  free(v);
  return rc;
}

/* ------------------------------------------------------------------------------------------
 * Three-dimensional extension (Sec. 2 calls it straightforward; Sec. 6.3 uses a 3-D specimen).
 * Voxel (x, y, z) of a W x H x D periodic volume is vol[(z*H + y)*W + x].
 *
 * Digitised segment from (0,0,0) to (dx,dy,dz): n = max(|dx|,|dy|,|dz|); the major axis is x
 * when |dx| = n, else y when |dy| = n, else z; k = 0..n along it, and every minor coordinate m
 * follows reading R1 on its own: sgn(m) floor((2k|m| + n) / (2n)), kept as an error term that
 * starts at n, grows by 2|m| per major step and steps when it reaches 2n.  With dz = 0 this is
 * oracle_bresenham.  Returns n + 1.
 * ------------------------------------------------------------------------------------------ */
int oracle_bresenham3(int dx, int dy, int dz, int *px, int *py, int *pz) {
  int a[3] = {dx < 0 ? -dx : dx, dy < 0 ? -dy : dy, dz < 0 ? -dz : dz};
  int sg[3] = {dx < 0 ? -1 : 1, dy < 0 ? -1 : 1, dz < 0 ? -1 : 1};
  int n = a[0];
  if (a[1] > n) n = a[1];
  if (a[2] > n) n = a[2];
  int major = a[0] == n ? 0 : (a[1] == n ? 1 : 2);
  long err[3] = {n, n, n};
  int c[3] = {0, 0, 0};
  for (int k = 0; k <= n; ++k) {
    if (k > 0) {
      for (int ax = 0; ax < 3; ++ax) {
        if (ax == major) {
          c[ax] = k;
          continue;
        }
        err[ax] += 2L * a[ax];
        if (err[ax] >= 2L * n) {
          err[ax] -= 2L * n;
          c[ax] += 1;
        }
      }
    }
    px[k] = sg[0] * c[0];
    py[k] = sg[1] * c[1];
    pz[k] = sg[2] * c[2];
  }
  return n + 1;
}

/* Canonical half of the 3-D cutoff box (one of each {v, -v}): the 2-D half domain at dz = 0 in
 * its own order, then for dz = 1..cz the rectangle [-cx,cx] x [-cy,cy] row by row (dy outer). */
int64_t oracle_num_vectors3(int cx, int cy, int cz) {
  return oracle_num_vectors(cx, cy) + (int64_t)cz * (2 * cx + 1) * (2 * cy + 1);
}

int oracle_vectors3(int cx, int cy, int cz, int16_t *v) {
  if (cx < 0 || cy < 0 || cz < 0) return -22;
  int64_t n2 = oracle_num_vectors(cx, cy);
  int16_t *t = (int16_t *)malloc(sizeof(int16_t) * 2 * n2);
  oracle_vectors(cx, cy, t);
  int64_t i = 0;
  for (int64_t j = 0; j < n2; ++j, ++i) {
    v[3 * i] = t[2 * j];
    v[3 * i + 1] = t[2 * j + 1];
    v[3 * i + 2] = 0;
  }
  free(t);
  for (int dz = 1; dz <= cz; ++dz)
    for (int dy = -cy; dy <= cy; ++dy)
      for (int dx = -cx; dx <= cx; ++dx, ++i) {
        v[3 * i] = (int16_t)dx;
        v[3 * i + 1] = (int16_t)dy;
        v[3 * i + 2] = (int16_t)dz;
      }
  return 0;
}

/* L_p(v) of a periodic volume for an explicit list of 3-D vectors (|dx| <= W-1, |dy| <= H-1,
 * |dz| <= D-1): counts[p][i], phase 0 first; the loops of Alg. "L2_eval" with one more
 * coordinate. */
int oracle_lpf3_vectors(const uint8_t *vol, int W, int H, int D, const int16_t *v, int64_t nv,
                        unsigned phase_mask, uint32_t *counts, int nthreads) {
  if (W < 1 || H < 1 || D < 1 || nv < 0) return -22;
  if (!phase_mask || (phase_mask & ~3u)) return -22;
  int maxlen = 1;
  for (int64_t i = 0; i < nv; ++i) {
    int a0 = abs(v[3 * i]), a1 = abs(v[3 * i + 1]), a2 = abs(v[3 * i + 2]);
    if (a0 > W - 1 || a1 > H - 1 || a2 > D - 1) return -22;
    if (a0 + 1 > maxlen) maxlen = a0 + 1;
    if (a1 + 1 > maxlen) maxlen = a1 + 1;
    if (a2 + 1 > maxlen) maxlen = a2 + 1;
  }
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel
  {
    int *px = (int *)malloc(sizeof(int) * maxlen);
    int *py = (int *)malloc(sizeof(int) * maxlen);
    int *pz = (int *)malloc(sizeof(int) * maxlen);
#pragma omp for schedule(dynamic, 4)
    for (int64_t i = 0; i < nv; ++i) {
      int np = oracle_bresenham3(v[3 * i], v[3 * i + 1], v[3 * i + 2], px, py, pz);
      int p = 0;
      for (int ph = 0; ph < 2; ++ph) {
        if (!(phase_mask & (1u << ph))) continue;
        uint32_t count = 0;
        for (int z = 0; z < D; ++z)
          for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
              int k;
              for (k = 0; k < np; ++k) {
                size_t q = ((size_t)wrap(z + pz[k], D) * H + wrap(y + py[k], H)) * W +
                           wrap(x + px[k], W);
                if (vol[q] != ph) break;
              }
              if (k == np) count += 1;
            }
        counts[(size_t)p * nv + i] = count;
        ++p;
      }
    }
    free(px);
    free(py);
    free(pz);
  }
  return 0;
}

/* The same over the canonical 3-D half domain. */
int oracle_lpf3(const uint8_t *vol, int W, int H, int D, int cx, int cy, int cz,
                unsigned phase_mask, uint32_t *counts, int nthreads) {
  if (W < 1 || H < 1 || D < 1 || cx < 0 || cy < 0 || cz < 0 || cx > W - 1 || cy > H - 1 ||
      cz > D - 1)
    return -22;
  int64_t nv = oracle_num_vectors3(cx, cy, cz);
  int16_t *v = (int16_t *)malloc(sizeof(int16_t) * 3 * nv);
  oracle_vectors3(cx, cy, cz, v);
  int rc = oracle_lpf3_vectors(vol, W, H, D, v, nv, phase_mask, counts, nthreads);
  free(v);
  return rc;
}

/* ------------------------------------------------------------------------------------------
 * Pixel interchange (Sec. 4): I' equals I with the values of pixels a and b exchanged
 * (linear indices y*W + x).  delta[s][p][i] = L_p(I')(v_i) - L_p(I)(v_i).
 * ------------------------------------------------------------------------------------------ */
int oracle_delta_swap_full(const uint8_t *img, int W, int H, int cx, int cy, unsigned phase_mask,
                           const int32_t *swaps, int n, int32_t *delta, int nthreads) {
  if (W < 1 || H < 1 || cx < 0 || cy < 0 || cx > W - 1 || cy > H - 1) return -22;
  int64_t nv = oracle_num_vectors(cx, cy);
  int nph = (phase_mask & 1) + ((phase_mask >> 1) & 1);
  size_t N = (size_t)W * H;
  uint8_t *img2 = (uint8_t *)malloc(N);
  uint32_t *c0 = (uint32_t *)malloc(sizeof(uint32_t) * nph * nv);
  uint32_t *c1 = (uint32_t *)malloc(sizeof(uint32_t) * nph * nv);
  int rc = oracle_lpf(img, W, H, cx, cy, phase_mask, 0, c0, nthreads);
  for (int s = 0; s < n && rc == 0; ++s) {
    int32_t a = swaps[2 * s], b = swaps[2 * s + 1];
    if (a < 0 || b < 0 || (size_t)a >= N || (size_t)b >= N) {
      rc = -22;
      break;
    }
    memcpy(img2, img, N);
    uint8_t t = img2[a];
    img2[a] = img2[b];
    img2[b] = t;
    rc = oracle_lpf(img2, W, H, cx, cy, phase_mask, 0, c1, nthreads);
    for (int64_t j = 0; j < (int64_t)nph * nv; ++j)
      delta[(size_t)s * nph * nv + j] = (int32_t)c1[j] - (int32_t)c0[j];
  }
  free(img2);
  free(c0);
  free(c1);
  return rc;
}

/* lambda(x) on the image I with pixels a and b interchanged (or on I itself when a < 0). */
static inline int seg_in_phase(const uint8_t *img, int W, int H, int x, int y, const int *px,
                               const int *py, int np, uint8_t phase, int a, int b) {
  for (int k = 0; k < np; ++k) {
    int xx = wrap(x + px[k], W), yy = wrap(y + py[k], H);
    int q = yy * W + xx;
    uint8_t val = img[q];
    if (a >= 0) {
      if (q == a) val = img[b];
      else if (q == b) val = img[a];
    }
    if (val != phase) return 0;
  }
  return 1;
}

/* Restricted recount: only translations whose segment covers a or b can change, so
 * delta = sum over x in (P_a u P_b) of [lambda(x; I') - lambda(x; I)], P_a = {a - p_k}. */
static void delta_one(const uint8_t *img, int W, int H, const int *px, const int *py, int np,
                      int a, int b, unsigned phase_mask, const uint8_t *sample /* or NULL */,
                      int32_t *out /* [nph] */) {
  int ax = a % W, ay = a / W, bx = b % W, by = b / W;
  int p = 0;
  for (int ph = 0; ph < 2; ++ph) {
    if (!(phase_mask & (1u << ph))) continue;
    int32_t d = 0;
    if (a != b && img[a] != img[b]) {
      for (int src = 0; src < 2; ++src) {
        int cxp = src ? bx : ax, cyp = src ? by : ay;
        for (int k = 0; k < np; ++k) {
          int x = wrap(cxp - px[k], W), y = wrap(cyp - py[k], H);
          if (src == 1) {
            /* skip translations already visited through a */
            int dup = 0;
            for (int j = 0; j < np && !dup; ++j)
              if (wrap(x + px[j], W) == ax && wrap(y + py[j], H) == ay) dup = 1;
            if (dup) continue;
          }
          if (sample && !sample[(size_t)y * W + x]) continue;  /* x not in the position set */
          d += seg_in_phase(img, W, H, x, y, px, py, np, (uint8_t)ph, a, b) -
               seg_in_phase(img, W, H, x, y, px, py, np, (uint8_t)ph, -1, -1);
        }
      }
    }
    out[p++] = d;
  }
}

static int delta_swap_impl(const uint8_t *img, int W, int H, int cx, int cy, unsigned phase_mask,
                           const int32_t *swaps, int n, const uint8_t *sample, int32_t *delta,
                           int nthreads) {
  if (W < 1 || H < 1 || cx < 0 || cy < 0 || cx > W - 1 || cy > H - 1) return -22;
  if (!phase_mask || (phase_mask & ~3u)) return -22;
  int64_t nv = oracle_num_vectors(cx, cy);
  int nph = (phase_mask & 1) + ((phase_mask >> 1) & 1);
  size_t N = (size_t)W * H;
  for (int s = 0; s < n; ++s)
    if (swaps[2 * s] < 0 || swaps[2 * s + 1] < 0 || (size_t)swaps[2 * s] >= N ||
        (size_t)swaps[2 * s + 1] >= N)
      return -22;
  int16_t *v = (int16_t *)malloc(sizeof(int16_t) * 2 * nv);
  oracle_vectors(cx, cy, v);
  int maxlen = (cx > cy ? cx : cy) + 1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel
  {
    int *px = (int *)malloc(sizeof(int) * maxlen);
    int *py = (int *)malloc(sizeof(int) * maxlen);
    int32_t tmp[2];
#pragma omp for schedule(dynamic, 1) collapse(2)
    for (int s = 0; s < n; ++s)
      for (int64_t i = 0; i < nv; ++i) {
        int np = oracle_bresenham(v[2 * i], v[2 * i + 1], px, py);
        delta_one(img, W, H, px, py, np, swaps[2 * s], swaps[2 * s + 1], phase_mask, sample, tmp);
        for (int p = 0; p < nph; ++p) delta[((size_t)s * nph + p) * nv + i] = tmp[p];
      }
    free(px);
    free(py);
  }
  free(v);
  return 0;
}

int oracle_delta_swap(const uint8_t *img, int W, int H, int cx, int cy, unsigned phase_mask,
                      const int32_t *swaps, int n, int32_t *delta, int nthreads) {
  return delta_swap_impl(img, W, H, cx, cy, phase_mask, swaps, n, NULL, delta, nthreads);
}

/* The change of the sampled counts (oracle_lpf_sampled) under pixel interchanges: the restricted
 * recount over the placements through a or b that lie in the position set. */
int oracle_delta_swap_sampled(const uint8_t *img, int W, int H, int cx, int cy,
                              unsigned phase_mask, const uint8_t *sample, const int32_t *swaps,
                              int n, int32_t *delta, int nthreads) {
  return delta_swap_impl(img, W, H, cx, cy, phase_mask, swaps, n, sample, delta, nthreads);
}

/* ------------------------------------------------------------------------------------------
 * S2 change under a pixel interchange (Sec. 4 operator applied to eq. (S2dis)):
 * delta[s][p][i] = C_p(I')(v_i) - C_p(I)(v_i) over the canonical half domain.  Only the pairs
 * (x, x + v) that contain a or b can change, i.e. the start pixels x in {a, b, a - v, b - v};
 * each distinct start pixel is counted once, before and after the interchange.
 * ------------------------------------------------------------------------------------------ */
static inline uint8_t pix_swapped(const uint8_t *img, int q, int a, int b) {
  if (q == a) return img[b];
  if (q == b) return img[a];
  return img[q];
}

int oracle_s2_delta_swap(const uint8_t *img, int W, int H, int cx, int cy, unsigned phase_mask,
                         const int32_t *swaps, int n, int32_t *delta, int nthreads) {
  if (W < 1 || H < 1 || cx < 0 || cy < 0 || cx > W - 1 || cy > H - 1) return -22;
  if (!phase_mask || (phase_mask & ~3u)) return -22;
  int64_t nv = oracle_num_vectors(cx, cy);
  int nph = (phase_mask & 1) + ((phase_mask >> 1) & 1);
  size_t N = (size_t)W * H;
  for (int s = 0; s < n; ++s)
    if (swaps[2 * s] < 0 || swaps[2 * s + 1] < 0 || (size_t)swaps[2 * s] >= N ||
        (size_t)swaps[2 * s + 1] >= N)
      return -22;
  int16_t *v = (int16_t *)malloc(sizeof(int16_t) * 2 * nv);
  oracle_vectors(cx, cy, v);
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 1) collapse(2)
  for (int s = 0; s < n; ++s)
    for (int64_t i = 0; i < nv; ++i) {
      int a = swaps[2 * s], b = swaps[2 * s + 1];
      int dx = v[2 * i], dy = v[2 * i + 1];
      int start[4];
      int ns = 0;
      int cand[4] = {a, b, wrap(a % W - dx, W) + wrap(a / W - dy, H) * W,
                     wrap(b % W - dx, W) + wrap(b / W - dy, H) * W};
      for (int j = 0; j < 4; ++j) {
        int seen = 0;
        for (int t = 0; t < ns; ++t) seen |= start[t] == cand[j];
        if (!seen) start[ns++] = cand[j];
      }
      int p = 0;
      for (int ph = 0; ph < 2; ++ph) {
        if (!(phase_mask & (1u << ph))) continue;
        int32_t d = 0;
        for (int t = 0; t < ns; ++t) {
          int x = start[t];
          int y = wrap(x / W + dy, H) * W + wrap(x % W + dx, W);
          d += (pix_swapped(img, x, a, b) == ph && pix_swapped(img, y, a, b) == ph) -
               (img[x] == ph && img[y] == ph);
        }
        delta[((size_t)s * nph + p) * nv + i] = d;
        ++p;
      }
    }
  free(v);
  return 0;
}

/* ------------------------------------------------------------------------------------------
 * Philox-4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of the 4-word Philox S-box
 * with multipliers 0xD2E7470EE14C6C93 / 0xCA5A826395121157 and Weyl key increments
 * 0x9E3779B97F4A7C15 / 0xBB67AE8584CAA73B.
 * ------------------------------------------------------------------------------------------ */
void oracle_philox4x64(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4]) {
  uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint64_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; ++r) {
    unsigned __int128 p0 = (unsigned __int128)0xD2E7470EE14C6C93ULL * c0;
    unsigned __int128 p1 = (unsigned __int128)0xCA5A826395121157ULL * c2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
    k0 += 0x9E3779B97F4A7C15ULL;
    k1 += 0xBB67AE8584CAA73BULL;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* ------------------------------------------------------------------------------------------
 * Simulated annealing with the least-square objective (Sec. 4, Alg. "annealing", eq. (LSE)).
 *
 * Objective: e = sum over phases p in the mask and vectors v of the canonical half domain of
 *   (T_p(v)/Nt - L_p(v)/N)^2, with T the target's exact counts over Nt pixels and N = W*H.
 * One step evaluates K candidate interchanges against the current state, in candidate order,
 * and applies the first one that passes the Metropolis test (rejections leave the state
 * unchanged, so this is the sequential chain with the later candidates of the step unused).
 *
 * Candidate k of step s: (r0,r1,r2,r3) = Philox4x64-10(ctr = {s, k, 0, 0}, key = {seed, 0x6c7066});
 *   a = pos1[((r0 >> 32) * n1) >> 32], b = pos0[((r1 >> 32) * n0) >> 32], U = (r2 >> 11) * 2^-53.
 *   pos1 / pos0 list the phase-1 / phase-0 pixels, initially in ascending index order; an
 *   accepted interchange writes b into a's slot of pos1 and a into b's slot of pos0.
 *   proposal 1 (interfacial pixels, reading R13): the candidate is void unless both a and b
 *   have a periodic 4-neighbour of the other phase.
 * Energy change, exact in integers:  S = sum dL * (Nt * (dL + 2 L) - 2 N T),
 *   de = (double)S / ((double)N * (double)N * (double)Nt).
 * Acceptance: de <= 0 or U < exp(-de / T_s).
 *
 * Ranked evaluation (reading R18 of the learned proposal; the paper leaves the operator open,
 * Sec. 4): given a per-pixel score field, the step still draws the same K candidates, but
 * evaluates first the min(64, R) draws with the largest fp32 key score[a] + score[b] among the
 * first R = min(K, 4096) draws (largest first, equal keys by draw index; a void draw or a NaN key
 * counts as -infinity), then every other draw in draw order; the first of this order that
 * passes the Metropolis test is applied, and its draw index is recorded.
 * ------------------------------------------------------------------------------------------ */
typedef struct {
  int32_t k, a, b;
  int32_t pad;
  double de, e;
} oracle_step_result;

static int interfacial(const uint8_t *img, int W, int H, int q) {
  int x = q % W, y = q / W;
  uint8_t v = img[q];
  return img[y * W + wrap(x + 1, W)] != v || img[y * W + wrap(x - 1, W)] != v ||
         img[wrap(y + 1, H) * W + x] != v || img[wrap(y - 1, H) * W + x] != v;
}

double oracle_lse(const uint32_t *counts, const uint32_t *target, int64_t nterms, int64_t N,
                  int64_t Nt) {
  double e = 0.0;
  for (int64_t j = 0; j < nterms; ++j) {
    double d = (double)((int64_t)N * (int64_t)target[j] - (int64_t)Nt * (int64_t)counts[j]);
    e += d * d;
  }
  return e / ((double)N * (double)N * (double)Nt * (double)Nt);
}

/* descriptor 0: the lineal path function (counts = L); descriptor 1: the two-point probability
 * (counts = W H S2, Sec. 2.1), the descriptor the paper compares against in Secs. 5 and 6.1. */
/* sample (LPF only): the Monte-Carlo position set of the cell; the counts are then sampled
 * counts and N in the objective is the number of sampled positions. */
/* The evaluation order of one step (ranked evaluation above): order[0..K). */
static void ranked_order(const int32_t *ca, const int32_t *cb, int K, const float *score,
                         int32_t *order, uint8_t *chosen) {
  int R = K < 4096 ? K : 4096;
  int top = R < 64 ? R : 64;
  for (int k = 0; k < K; ++k) chosen[k] = 0;
  for (int t = 0; t < top; ++t) {
    int best = -1;
    float best_key = 0.0f;
    for (int k = 0; k < R; ++k) {
      if (chosen[k]) continue;
      float key = -INFINITY;
      if (ca[k] >= 0 && cb[k] >= 0) {
        key = score[ca[k]] + score[cb[k]];
        if (isnan(key)) key = -INFINITY;
      }
      if (best < 0 || key > best_key) {
        best = k;
        best_key = key;
      }
    }
    chosen[best] = 1;
    order[t] = best;
  }
  int t = top;
  for (int k = 0; k < K; ++k)
    if (!chosen[k]) order[t++] = k;
}

static int anneal_core(uint8_t *img, int W, int H, int cx, int cy, unsigned phase_mask,
                       int descriptor, const uint8_t *sample, uint32_t *counts,
                       const uint32_t *target, int64_t Nt, uint64_t seed, uint64_t step0,
                       int nsteps, int K, const double *Ts, int proposal, const float *score,
                       int32_t *pos1, int32_t *pos0, double *e_io, oracle_step_result *res,
                       int nthreads) {
  if (W < 1 || H < 1 || cx < 0 || cy < 0 || cx > W - 1 || cy > H - 1 || K < 1) return -22;
  if (descriptor != 0 && descriptor != 1) return -22;
  if (sample && descriptor != 0) return -22;
  int64_t nv = oracle_num_vectors(cx, cy);
  int nph = (phase_mask & 1) + ((phase_mask >> 1) & 1);
  int64_t N = (int64_t)W * H;
  if (sample) {
    N = 0;
    for (int64_t q = 0; q < (int64_t)W * H; ++q) N += sample[q] != 0;
    if (N < 1) return -22;
  }
  int n1 = 0;
  for (int64_t q = 0; q < (int64_t)W * H; ++q) n1 += img[q] == 1;
  int n0 = W * H - n1;
  if (n1 == 0 || n0 == 0) return -22;
  int16_t *v = (int16_t *)malloc(sizeof(int16_t) * 2 * nv);
  oracle_vectors(cx, cy, v);
  int32_t *dl = (int32_t *)malloc(sizeof(int32_t) * nph * nv);
  int32_t sw[2];
  /* the step's draws: slots, pixels (a = -1 for a void draw) and uniforms */
  int32_t *cia = (int32_t *)malloc(sizeof(int32_t) * K), *cib = (int32_t *)malloc(sizeof(int32_t) * K);
  int32_t *ca = (int32_t *)malloc(sizeof(int32_t) * K), *cb = (int32_t *)malloc(sizeof(int32_t) * K);
  double *cu = (double *)malloc(sizeof(double) * K);
  int32_t *order = (int32_t *)malloc(sizeof(int32_t) * K);
  uint8_t *chosen = (uint8_t *)malloc(K);
  double e = *e_io;
  for (int s = 0; s < nsteps; ++s) {
    uint64_t step = step0 + (uint64_t)s;
    oracle_step_result r = {-1, -1, -1, 0, 0.0, e};
    for (int k = 0; k < K; ++k) {
      uint64_t ctr[4] = {step, (uint64_t)k, 0, 0}, key[2] = {seed, 0x6c7066ULL}, o[4];
      oracle_philox4x64(ctr, key, o);
      cia[k] = (int)(((o[0] >> 32) * (uint64_t)n1) >> 32);
      cib[k] = (int)(((o[1] >> 32) * (uint64_t)n0) >> 32);
      cu[k] = (double)(o[2] >> 11) * (1.0 / 9007199254740992.0);
      ca[k] = pos1[cia[k]];
      cb[k] = pos0[cib[k]];
      if (proposal == 1 && !(interfacial(img, W, H, ca[k]) && interfacial(img, W, H, cb[k])))
        ca[k] = cb[k] = -1;
    }
    if (score)
      ranked_order(ca, cb, K, score, order, chosen);
    else
      for (int k = 0; k < K; ++k) order[k] = k;
    for (int t = 0; t < K; ++t) {
      int k = order[t];
      int ia = cia[k], ib = cib[k], a = ca[k], b = cb[k];
      double U = cu[k];
      if (a < 0) continue;
      sw[0] = a;
      sw[1] = b;
      if (descriptor == 0)
        delta_swap_impl(img, W, H, cx, cy, phase_mask, sw, 1, sample, dl, nthreads);
      else
        oracle_s2_delta_swap(img, W, H, cx, cy, phase_mask, sw, 1, dl, nthreads);
      int64_t S = 0;
      for (int64_t j = 0; j < (int64_t)nph * nv; ++j) {
        int64_t d = dl[j];
        S += d * (Nt * (d + 2 * (int64_t)counts[j]) - 2 * N * (int64_t)target[j]);
      }
      double de = (double)S / ((double)N * (double)N * (double)Nt);
      if (de <= 0.0 || U < exp(-de / Ts[s])) {
        for (int64_t j = 0; j < (int64_t)nph * nv; ++j)
          counts[j] = (uint32_t)((int64_t)counts[j] + dl[j]);
        img[a] = 0;
        img[b] = 1;
        pos1[ia] = b;
        pos0[ib] = a;
        e += de;
        r.k = k;
        r.a = a;
        r.b = b;
        r.de = de;
        r.e = e;
        break;
      }
    }
    res[s] = r;
  }
  *e_io = e;
  free(v);
  free(dl);
  free(cia);
  free(cib);
  free(ca);
  free(cb);
  free(cu);
  free(order);
  free(chosen);
  return 0;
}

int oracle_anneal_run_desc(uint8_t *img, int W, int H, int cx, int cy, unsigned phase_mask,
                           int descriptor,
                           uint32_t *counts /* [nph][nv], must equal the descriptor of img */,
                           const uint32_t *target /* [nph][nv] */, int64_t Nt, uint64_t seed,
                           uint64_t step0, int nsteps, int K, const double *Ts /* [nsteps] */,
                           int proposal, int32_t *pos1, int32_t *pos0 /* in/out */,
                           double *e_io, oracle_step_result *res /* [nsteps] */, int nthreads) {
  return anneal_core(img, W, H, cx, cy, phase_mask, descriptor, NULL, counts, target, Nt, seed,
                     step0, nsteps, K, Ts, proposal, NULL, pos1, pos0, e_io, res, nthreads);
}

int oracle_anneal_run(uint8_t *img, int W, int H, int cx, int cy, unsigned phase_mask,
                      uint32_t *counts, const uint32_t *target, int64_t Nt, uint64_t seed,
                      uint64_t step0, int nsteps, int K, const double *Ts, int proposal,
                      int32_t *pos1, int32_t *pos0, double *e_io, oracle_step_result *res,
                      int nthreads) {
  return anneal_core(img, W, H, cx, cy, phase_mask, 0, NULL, counts, target, Nt, seed, step0,
                     nsteps, K, Ts, proposal, NULL, pos1, pos0, e_io, res, nthreads);
}

/* The chain with the ranked evaluation order over a fixed score field (score: float [W*H]). */
int oracle_anneal_run_ranked(uint8_t *img, int W, int H, int cx, int cy, unsigned phase_mask,
                             uint32_t *counts, const uint32_t *target, int64_t Nt,
                             uint64_t seed, uint64_t step0, int nsteps, int K, const double *Ts,
                             int proposal, const float *score, int32_t *pos1, int32_t *pos0,
                             double *e_io, oracle_step_result *res, int nthreads) {
  if (!score) return -22;
  return anneal_core(img, W, H, cx, cy, phase_mask, 0, NULL, counts, target, Nt, seed, step0,
                     nsteps, K, Ts, proposal, score, pos1, pos0, e_io, res, nthreads);
}

/* The chain driven by the Monte-Carlo approximation: counts = oracle_lpf_sampled of img over the
 * cell's position set `sample`, target = sampled counts of the original over Nt positions. */
int oracle_anneal_run_sampled(uint8_t *img, int W, int H, int cx, int cy, unsigned phase_mask,
                              const uint8_t *sample, uint32_t *counts, const uint32_t *target,
                              int64_t Nt, uint64_t seed, uint64_t step0, int nsteps, int K,
                              const double *Ts, int proposal, int32_t *pos1, int32_t *pos0,
                              double *e_io, oracle_step_result *res, int nthreads) {
  if (!sample) return -22;
  return anneal_core(img, W, H, cx, cy, phase_mask, 0, sample, counts, target, Nt, seed, step0,
                     nsteps, K, Ts, proposal, NULL, pos1, pos0, e_io, res, nthreads);
}
