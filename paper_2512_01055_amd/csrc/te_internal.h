// Internal interfaces between the C-ABI host code and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace te {

// Virtual dimensions are padded to a multiple of this in every device
// layout; padded entries are zero, so they add nothing to any contraction.
constexpr int VPAD = 8;
// Edge of the cubic boxes the W arrays are stored in: element (a,b,c) lives
// at ((A*nT + B)*nT + C)*BOX^3 + (a%BOX)*BOX^2 + (b%BOX)*BOX + c%BOX.
constexpr int BOX = 8;
constexpr int BOX3 = BOX * BOX * BOX;

inline int pad_v(int v) { return (v + VPAD - 1) / VPAD * VPAD; }

enum class Prec : int { F64 = 0, F32 = 1, BF16X3 = 2, BF16X2 = 3, FP16X2 = 4 };

// One occupied triple's W build: three GEMMs (one per lone virtual index),
// each M = vp^2 (virtual pairs) x N = vp (lone index) x K = 2 vp + 2 o.
struct WItem {
  const void *Xs[3];  // slices (ix|yf) for x in i, j, k: [vp][vp][vp] each;
                      // part p of slice q at Xs[q] + p * xps
  // t2 reached through panels of the occupied indices q_0, q_1, q_2 = i, j, k
  // (elements of the operand type; blocks are [vp][vp]):
  //   column panel   block t2[p][q_x] at Tc[x] + p * tcs
  //   row panel      block t2[q_x][l] at Tr[x] + l * trs   (FP64 / FP32 modes)
  //   row form       t_{q_x l}^{yz}  at Tt[x] + (y vp + z) lo + l (16-bit modes)
  // A resident t2 [part][o][o][vp][vp] gives tcs = o vp^2, trs = vp^2; panels
  // copied into a cache slot give tcs = trs = vp^2. Part p of a column panel
  // (or of the occupied segments' row panel) at + p * tcps, of the row form
  // at + p * t2tps.
  const void *Tc[3], *Tr[3], *Tt[3];
  const void *In;  // -(px|ql), layout [part][o][vp][o][lo]
  size_t xps, tcs, trs, tcps, ips, t2tps;
  int lo;          // length of the occupied rows of In and the row form: o in
                   // FP64 and FP32 modes, o rounded up to 8 (zero padded) in
                   // 16-bit modes
  void *W;         // three boxed W arrays of vp^3 each (FP64 or FP32)
  float scale;     // FP16 parts: 1 / (sigma_X sigma_T), applied to W; else 1
  int o, vp, i, j, k;
  int mt, nt;      // tiles along M and N
};

// One occupied triple's energy: sum over virtual box sextets.
struct EItem {
  const void *W;       // as written by the W build
  // (jb|kc), (ia|kc), (ia|jb) for this triple, each a v x v block with row
  // stride kld (views of the resident [o][vp][o][vp] array, or per-triple
  // blocks assembled from the factors)
  const double *Kjk, *Kik, *Kij;
  long kld;
  const double *t1;    // [o][vp]
  const double *eo;    // [o]
  const double *ev;    // [vp]
  const int *sext;     // packed box triples A>=B>=C: A | B<<10 | C<<20
  double *part;        // [nsext] partial sums of the W Z / D terms (E[4])
  double *part5;       // [nsext] partial sums of the V Z / D terms (E[5])
  int o, v, vp, nT, i, j, k, nsext;
};

// Per-triple reduction: S4 = sum(part[0..n)), S5 = sum(part5[0..n)), both in a
// fixed order; e = w (S4 + S5).
struct RItem {
  const double *part, *part5;
  double *out;          // w (S4 + S5)
  double *out4, *out5;  // w S4, w S5 (optional)
  int n;
  double w;
};

// Generic FP64 "TN" product used for staging:
//   C[row_off(m) + col_off(n)] = alpha * sum_q A[q*lda + m] * B[q*ldb + n]
// with off(x) = (x / d) * s1 + (x % d) * s2.
struct GemmTN {
  const double *A, *B;
  double *C;
  int M, N, K;
  long lda, ldb;
  int rd; long rs1, rs2;
  int cd; long cs1, cs2;
  double alpha;
};

// Launchers (W build in te_wbuild.hip, the rest in te_kernels.hip). All
// return the hipError_t of the launch.
// W-build tile shape: BM = 64 wm rows (virtual pairs), BN = 16 nb columns;
// wm = 2 is the only row count built.
struct WConfig {
  int nb = 5, wm = 2;
  int bm() const { return 64 * wm; }
  int bn() const { return 16 * nb; }
};
WConfig wbuild_config(Prec p, int vp);
hipError_t launch_wbuild(Prec p, const WItem *d_items, const int *d_tile_item, int nitems,
                         int tiles_per_item, long total_tiles, WConfig cfg, hipStream_t s);
hipError_t launch_energy(bool w_is_f64, const EItem *d_items, const int *d_blk_item,
                         int nitems, int blks_per_item, long total_blks, hipStream_t s);
hipError_t launch_reduce(const RItem *d_items, int nitems, hipStream_t s);
hipError_t launch_sum(const double *x, long n, double *out, hipStream_t s);
hipError_t launch_gemm_tn(const GemmTN &g, hipStream_t s);
// up to three independent products in one launch (one grid layer each)
hipError_t launch_gemm_tn_batch(const GemmTN *g, int n, hipStream_t s);
hipError_t launch_pad4(const double *src, double *dst, int d0, int d1, int d2, int d3,
                       int p1, int p2, int p3, double scale, hipStream_t s);
hipError_t launch_to_f32(const double *src, float *dst, size_t n, hipStream_t s);
hipError_t launch_to_bf16_parts(const double *src, uint16_t *dst, size_t n, int nparts,
                                hipStream_t s);
// BF16 parts of t2 [o][o][vp][vp] regrouped as [part][o][vp*vp][lo] (occupied
// index last, zero for l >= o).
// Column panel and row panel (FP64, FP32) or row form (16-bit parts) of one
// occupied index from its FP64 column panel [o][v][v]; see panel_kernel.
// sigma: the t2 scale of the FP16 parts (ignored otherwise).
hipError_t launch_panel(Prec p, const double *stg, void *col, void *row, int o, int v, int vp,
                        int lo, double sigma, hipStream_t s);
// Scaled FP16 parts (two, [2][n]) of sigma * x, in the layouts of the BF16
// launchers above; sigma is a power of two.
hipError_t launch_to_f16_parts(const double *src, uint16_t *dst, size_t n, double sigma,
                               hipStream_t s);
hipError_t launch_t2t_f16_parts(const double *t2, uint16_t *dst, int o, int vp, int lo,
                                double sigma, hipStream_t s);
hipError_t launch_in_f16_parts(const double *in, uint16_t *dst, int o, int vp, int lo,
                               double sigma, hipStream_t s);
// Max |x| (absmax) or max over columns of sum_Q B[Q][c]^2 (colnorm_max), into
// *out as the bits of a non-negative double; *out must start at 0.
hipError_t launch_absmax(const double *x, size_t n, unsigned long long *out, hipStream_t s);
hipError_t launch_colnorm_max(const double *B, int naux, long ncol, unsigned long long *out,
                              hipStream_t s);
hipError_t launch_t2t_bf16_parts(const double *t2, uint16_t *dst, int o, int vp, int lo,
                                 int nparts, hipStream_t s);
// BF16 parts of In [o][vp][o][o] with the last index padded to lo.
hipError_t launch_in_bf16_parts(const double *in, uint16_t *dst, int o, int vp, int lo,
                                int nparts, hipStream_t s);
hipError_t launch_check(const double *x, size_t n, int *flag, hipStream_t s);
hipError_t launch_mfma_probe(Prec p, void *out, int blocks, int iters, hipStream_t s,
                             double *flops);
hipError_t launch_t2_asym(const double *t2, int o, int v, double *maxdiff, double *maxabs,
                          hipStream_t s);

}  // namespace te
