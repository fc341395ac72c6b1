// W build of the (T) library for gfx950: W^{abc}_{ijk} of Eq. 2 summed over
// the pair permutations of Eq. 5, as three MFMA GEMMs per occupied triple (one
// per virtual index that stands alone in a term), with its launchers.
#include "te_device.h"

namespace te {
namespace {

// ------------------------------------------------------------ W build
//
// For triple (i,j,k) and lone index g (0: c, 1: a, 2: b) the kernel forms
//   C[m][n] = sum_f A0[m][f] B0[n][f] + sum_f A1[m][f] B1[n][f]
//           + sum_l A2[m][l] B2[n][l] + sum_l A3[m][l] B3[n][l]
// where m runs over the two paired virtual indices (vp^2) and n over the
// lone one. With X_p[x][y][f] = (px|yf), T_pq[z][f] = t_pq^zf,
// t_{l r}^{yz} = t2[l][r][y][z] and In_pq[x][l] = -(px|ql):
//   g=0 (lone c), m=(a,b): X_i[a][b]·T_kj[c] + X_j[b][a]·T_ki[c]
//                          + t_{il}^{ab}·In_kj[c] + t_{lj}^{ab}·In_ki[c]
//   g=1 (lone a), m=(b,c): X_j[b][c]·T_ik[a] + X_k[c][b]·T_ij[a]
//                          + t_{lk}^{bc}·In_ij[a] + t_{jl}^{bc}·In_ik[a]
//   g=2 (lone b), m=(a,c): X_i[a][c]·T_jk[b] + X_k[c][a]·T_ji[b]
//                          + t_{lk}^{ac}·In_ji[b] + t_{il}^{ac}·In_jk[b]
// These are the twelve terms of Eq. 2 under the six permutations of Eq. 5,
// grouped by the index that is not paired with another virtual index. The
// three results are written to separate boxed arrays; W is their sum.
// Occupied indices are named by value (tq, ix, iy) where they select a row,
// and by position in (i, j, k) (xa, tr, op) where they select a slice or a
// t2 panel.
struct Setup {
  int xa[2];      // X slice (0: X_i, 1: X_j, 2: X_k) of segments 0/1 (seg 1 transposed)
  int tq[2], tr[2];  // T_{tq tr} rows for the B side of segments 0/1 (tr: position)
  int op[2], om[2];  // occupied-term A side (op: position): om 0 -> t2[op][l], 1 -> t2[l][op]
  int ix[2], iy[2];  // In_{ix iy} rows for segments 2/3
};

__device__ inline Setup make_setup(int g, int i, int j, int k) {
  Setup s;
  if (g == 0) {
    s.xa[0] = 0; s.xa[1] = 1;
    s.tq[0] = k; s.tr[0] = 1; s.tq[1] = k; s.tr[1] = 0;
    s.op[0] = 0; s.om[0] = 0; s.op[1] = 1; s.om[1] = 1;
    s.ix[0] = k; s.iy[0] = j; s.ix[1] = k; s.iy[1] = i;
  } else if (g == 1) {
    s.xa[0] = 1; s.xa[1] = 2;
    s.tq[0] = i; s.tr[0] = 2; s.tq[1] = i; s.tr[1] = 1;
    s.op[0] = 2; s.om[0] = 1; s.op[1] = 1; s.om[1] = 0;
    s.ix[0] = i; s.iy[0] = j; s.ix[1] = i; s.iy[1] = k;
  } else {
    s.xa[0] = 0; s.xa[1] = 2;
    s.tq[0] = j; s.tr[0] = 2; s.tq[1] = j; s.tr[1] = 0;
    s.op[0] = 2; s.om[0] = 1; s.op[1] = 0; s.om[1] = 0;
    s.ix[0] = j; s.iy[0] = i; s.ix[1] = j; s.iy[1] = k;
  }
  return s;
}

// NB: 16-column blocks per tile (BN = 16 NB); WM: 16-row blocks per wave
// (BM = 4 waves x 16 WM rows). The register budget asks for three waves per
// SIMD. The two LDS stages hold 2 NP (BM + BN) KT elements: 52 KiB at
// BM = 128, BN = 80 for FP64, FP32 and the two-part 16-bit modes, so three
// workgroups share a CU's 160 KiB; three BF16 parts (78 KiB) fit two.
template <Prec P, int NB, int WM>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(3))) void wbuild_kernel(const WItem *__restrict__ items,
                                                    const int *__restrict__ tile_item,
                                                    int tiles_per_item, long total_tiles) {
  using TR = Tr<P>;
  using T = typename TR::T;
  using Acc = typename TR::Acc;
  using Out = typename TR::Out;
  constexpr int KT = TR::KT, LD = TR::KT + TR::PAD, NP = TR::NP, KM = TR::KM;
  constexpr int BN = 16 * NB;
  constexpr int BM = 64 * WM;
  constexpr int CPR = KT / 8;                     // 8-element chunks per row
  constexpr int CA = (BM * KT / 8 + WG - 1) / WG; // A chunks per thread
  constexpr int CB = (BN * KT / 8 + WG - 1) / WG; // B chunks per thread

  __shared__ __attribute__((aligned(16))) T As[2][NP][BM][LD];
  __shared__ __attribute__((aligned(16))) T Bs[2][NP][BN][LD];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;

  // tile_item (mixed launches): [total_tiles] item of each tile, then
  // [nitems] first tile of each item. Without it every item has
  // tiles_per_item tiles.
  const long logical = xcd_remap(blockIdx.x, total_tiles);
  int it;
  long local;
  if (tile_item) {
    it = tile_item[logical];
    local = logical - tile_item[total_tiles + it];
  } else {
    it = (int)(logical / tiles_per_item);
    local = logical - (long)it * tiles_per_item;
  }
  const WItem &w = items[it];
  const int o = w.o, vp = w.vp, mt = w.mt, nt = w.nt;
  const int per_g = mt * nt;
  const int g = (int)(local / per_g);
  const int rr = (int)(local - (long)g * per_g);
  const int m0 = (rr / nt) * BM;
  const int n0 = (rr % nt) * BN;
  const long M = (long)vp * vp;
  const long vp2 = M;

  const Setup su = make_setup(g, w.i, w.j, w.k);
  const T *XA0 = reinterpret_cast<const T *>(w.Xs[su.xa[0]]);
  const T *XA1 = reinterpret_cast<const T *>(w.Xs[su.xa[1]]);
  const T *In = reinterpret_cast<const T *>(w.In);
  // t2 through the panels of i, j, k: T_{tq tr} rows of the X segments, and
  // the occupied segments' t2[op][l] (row panel) or t2[l][op] (column panel)
  const T *TB0 = reinterpret_cast<const T *>(w.Tc[su.tr[0]]) + (long)su.tq[0] * w.tcs;
  const T *TB1 = reinterpret_cast<const T *>(w.Tc[su.tr[1]]) + (long)su.tq[1] * w.tcs;

  // --- per-thread row pointers for the X phase
  long rowA[CA][2];
  int  kcA[CA];
  bool okA[CA];
#pragma unroll
  for (int u = 0; u < CA; ++u) {
    int c = tid + u * WG;
    int row = c / CPR;
    kcA[u] = (c % CPR) * 8;
    long m = m0 + row;
    okA[u] = (c < BM * CPR) && (m < M);
    long mm = okA[u] ? m : 0;
    long mx = mm / vp, my = mm - mx * vp;
    rowA[u][0] = mm * vp;
    rowA[u][1] = (my * vp + mx) * vp;
  }
  long rowB[CB];
  long rowI[CB][2];
  int kcB[CB];
  bool okB[CB];
#pragma unroll
  for (int u = 0; u < CB; ++u) {
    int c = tid + u * WG;
    int row = c / CPR;
    kcB[u] = (c % CPR) * 8;
    int n = n0 + row;
    okB[u] = (c < BN * CPR) && (n < vp);
    long nn = okB[u] ? n : 0;
    rowB[u] = nn * vp;
  }
  const T *TO[2];
  long ksO[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    if (su.om[s] == 0) { TO[s] = reinterpret_cast<const T *>(w.Tr[su.op[s]]); ksO[s] = (long)w.trs; }
    else               { TO[s] = reinterpret_cast<const T *>(w.Tc[su.op[s]]); ksO[s] = (long)w.tcs; }
  }
  // 16-bit modes: occupied-segment rows of T2T (t_{p l}^{yz} with l last), read
  // like the X rows; om = 1 takes the swapped pair (t_{l p}^{yz} = t_{p l}^{zy})
  const int lo = w.lo;
  const T *TT0 = reinterpret_cast<const T *>(w.Tt[su.op[0]]);
  const T *TT1 = reinterpret_cast<const T *>(w.Tt[su.op[1]]);
  long rowO[TR::SPLIT ? CA : 1][2];
  if constexpr (TR::SPLIT) {
#pragma unroll
    for (int u = 0; u < CA; ++u) {
      long mm = okA[u] ? (long)m0 + (tid + u * WG) / CPR : 0;
      long mx = mm / vp, my = mm - mx * vp;
#pragma unroll
      for (int s = 0; s < 2; ++s)
        rowO[u][s] = (su.om[s] ? my * vp + mx : mm) * lo;
    }
  }
#pragma unroll
  for (int u = 0; u < CB; ++u) {   // In rows have length lo
    long nn = okB[u] ? (long)n0 + (tid + u * WG) / CPR : 0;
    rowI[u][0] = (((long)su.ix[0] * vp + nn) * o + su.iy[0]) * lo;
    rowI[u][1] = (((long)su.ix[1] * vp + nn) * o + su.iy[1]) * lo;
  }

  const int KX = 2 * vp;
  const int KO = TR::SPLIT ? 2 * lo : 2 * o;
  const int nkx = (KX + KT - 1) / KT;
  const int nko = (KO + KT - 1) / KT;
  const int ntiles = nkx + nko;

  Chunk<T> ra[CA][NP], rb[CB][NP];

  auto load = [&](int t) {
    if (t < nkx) {
      const int kb = t * KT;
#pragma unroll
      for (int u = 0; u < CA; ++u) {
        int kg = kb + kcA[u];
        bool ok = okA[u] && kg < KX;
        int seg = kg >= vp;
        long off = rowA[u][seg] + (kg - seg * vp);
        const T *xb = seg ? XA1 : XA0;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          if (ok) ra[u][p].load(xb + p * w.xps + off); else ra[u][p].zero();
        }
      }
#pragma unroll
      for (int u = 0; u < CB; ++u) {
        int kg = kb + kcB[u];
        bool ok = okB[u] && kg < KX;
        int seg = kg >= vp;
        long off = rowB[u] + (kg - seg * vp);
        const T *tb = seg ? TB1 : TB0;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          if (ok) rb[u][p].load(tb + p * w.tcps + off); else rb[u][p].zero();
        }
      }
    } else if constexpr (TR::SPLIT) {
      // occupied segments as 8-element chunks of K-contiguous rows
      const int kb = (t - nkx) * KT;
#pragma unroll
      for (int u = 0; u < CA; ++u) {
        int kg = kb + kcA[u];
        bool ok = okA[u] && kg < KO;
        int seg = kg >= lo;
        long off = rowO[u][seg] + (kg - seg * lo);
        const T *tt = seg ? TT1 : TT0;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          if (ok) ra[u][p].load(tt + p * w.t2tps + off); else ra[u][p].zero();
        }
      }
#pragma unroll
      for (int u = 0; u < CB; ++u) {
        int kg = kb + kcB[u];
        bool ok = okB[u] && kg < KO;
        int seg = kg >= lo;
        long off = rowI[u][seg] + (kg - seg * lo);
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          if (ok) rb[u][p].load(In + p * w.ips + off); else rb[u][p].zero();
        }
      }
    } else {
      // K-major A: thread c takes k = c % KT and eight consecutive m, so the
      // transposed LDS stores of a lane group fill one row (conflict-free)
      const int kb = (t - nkx) * KT;
#pragma unroll
      for (int u = 0; u < CA; ++u) {
        int c = tid + u * WG;
        int kk = c % KT;
        int mc = (c / KT) * 8;
        int kg = kb + kk;
        long m = m0 + mc;
        bool ok = (c < BM * CPR) && kg < KO && m < M;
        int seg = kg >= o;
        long off = (long)(kg - seg * o) * ksO[seg] + m;
        const T *to = seg ? TO[1] : TO[0];
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          if (ok) ra[u][p].load(to + p * w.tcps + off); else ra[u][p].zero();
        }
      }
#pragma unroll
      for (int u = 0; u < CB; ++u) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          int kg = kb + kcB[u] + e;
          bool ok = okB[u] && kg < KO;
          int seg = kg >= o;
          long off = rowI[u][seg] + (kg - seg * o);
#pragma unroll
          for (int p = 0; p < NP; ++p) rb[u][p].set(e, ok ? gld(In + p * w.ips + off) : T(0));
        }
      }
    }
  };

  auto store = [&](int t, int buf) {
    if (t < nkx || TR::SPLIT) {
#pragma unroll
      for (int u = 0; u < CA; ++u) {
        int c = tid + u * WG;
        if (c < BM * CPR) {
          int row = c / CPR;
#pragma unroll
          for (int p = 0; p < NP; ++p) store_chunk<TR>(&As[buf][p][row][0], row, kcA[u], ra[u][p]);
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < CA; ++u) {
        int c = tid + u * WG;
        if (c < BM * CPR) {
          int kk = c % KT;
          int mc = (c / KT) * 8;
#pragma unroll
          for (int p = 0; p < NP; ++p)
#pragma unroll
            for (int e = 0; e < 8; ++e) As[buf][p][mc + e][lcol<TR>(mc + e, kk)] = ra[u][p].get(e);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < CB; ++u) {
      int c = tid + u * WG;
      if (c < BN * CPR) {
        int row = c / CPR;
#pragma unroll
        for (int p = 0; p < NP; ++p) store_chunk<TR>(&Bs[buf][p][row][0], row, kcB[u], rb[u][p]);
      }
    }
  };

  Acc acc[WM][NB];
#pragma unroll
  for (int a = 0; a < WM; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[a][b][r] = 0;

  const int wrow = wave * 16 * WM;
  const int fr = lane & 15;
  const int fk = lane >> 4;

  load(0);
  store(0, 0);
  __syncthreads();
  for (int t = 0; t < ntiles; ++t) {
    const int cur = t & 1;
    if (t + 1 < ntiles) load(t + 1);
#pragma unroll
    for (int kk = 0; kk < KT / KM; ++kk) {
      if constexpr (NP == 1) {
        using E = T;
        E av[WM], bv[NB];
#pragma unroll
        for (int rb_ = 0; rb_ < WM; ++rb_) {
          const int r = wrow + rb_ * 16 + fr;
          av[rb_] = As[cur][0][r][lcol<TR>(r, kk * 4 + fk)];
        }
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) bv[cb] = Bs[cur][0][cb * 16 + fr][lcol<TR>(cb * 16 + fr, kk * 4 + fk)];
#pragma unroll
        for (int rb_ = 0; rb_ < WM; ++rb_)
#pragma unroll
          for (int cb = 0; cb < NB; ++cb) acc[rb_][cb] = mma(av[rb_], bv[cb], acc[rb_][cb]);
      } else {
        using F = typename TR::Frag;
        F av[WM][NP], bv[NB][NP];
#pragma unroll
        for (int rb_ = 0; rb_ < WM; ++rb_)
#pragma unroll
          for (int p = 0; p < NP; ++p)
            av[rb_][p] = *reinterpret_cast<const F *>(
                &As[cur][p][wrow + rb_ * 16 + fr][lcol<TR>(wrow + rb_ * 16 + fr, fk * 8)]);
#pragma unroll
        for (int cb = 0; cb < NB; ++cb)
#pragma unroll
          for (int p = 0; p < NP; ++p)
            bv[cb][p] = *reinterpret_cast<const F *>(&Bs[cur][p][cb * 16 + fr][lcol<TR>(cb * 16 + fr, fk * 8)]);
#pragma unroll
        for (int rb_ = 0; rb_ < WM; ++rb_)
#pragma unroll
          for (int cb = 0; cb < NB; ++cb) {
            // smallest cross products first: sum over pa + pb < NP
#pragma unroll
            for (int s = NP - 1; s >= 0; --s)
#pragma unroll
              for (int pa = s; pa >= 0; --pa)
                acc[rb_][cb] = mma(av[rb_][pa], bv[cb][s - pa], acc[rb_][cb]);
          }
      }
    }
    if (t + 1 < ntiles) store(t + 1, cur ^ 1);
    __syncthreads();
  }

  // epilogue: boxed store of this GEMM's share of W
  Out *Wg = reinterpret_cast<Out *>(w.W) + (long)g * vp2 * vp;
  const int nT = vp >> 3;
#pragma unroll
  for (int rb_ = 0; rb_ < WM; ++rb_)
#pragma unroll
    for (int cb = 0; cb < NB; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        long m = m0 + wrow + rb_ * 16 + (TR::ROWQ == 1 ? fk + 4 * r : fk * 4 + r);
        int n = n0 + cb * 16 + fr;
        if (m < M && n < vp) {
          int p0 = (int)(m / vp), p1 = (int)(m - (long)p0 * vp);
          int a, b, c;
          if (g == 0) { a = p0; b = p1; c = n; }
          else if (g == 1) { a = n; b = p0; c = p1; }
          else { a = p0; b = n; c = p1; }
          Out x = (Out)acc[rb_][cb][r];
          if constexpr (TR::SCALED) x *= w.scale;
          gst(Wg + box_off(a, b, c, nT), x);
        }
      }
}

}  // namespace

// ------------------------------------------------------------ launchers
// Tile shape: two 16-row blocks per wave in every precision, and the
// column-block count NB in [4, 8] that minimises padded waste of the lone
// index (larger NB on ties).
WConfig wbuild_config(Prec, int vp) {
  WConfig c;
  c.wm = 2;
  int best = 8;
  long best_w = -1;
  for (int nb = 8; nb >= 4; --nb) {
    int bn = 16 * nb;
    long tiles = (vp + bn - 1) / bn;
    long waste = tiles * bn - vp;
    if (best_w < 0 || waste < best_w) { best_w = waste; best = nb; }
  }
  c.nb = best;
  return c;
}

template <Prec P, int WM>
static hipError_t launch_wb_pw(const WItem *d_items, const int *d_tile_item, int tiles_per_item,
                               long total, int nb, hipStream_t s) {
  dim3 grid((unsigned)total), block(WG);
  switch (nb) {
    case 4: wbuild_kernel<P, 4, WM><<<grid, block, 0, s>>>(d_items, d_tile_item, tiles_per_item, total); break;
    case 5: wbuild_kernel<P, 5, WM><<<grid, block, 0, s>>>(d_items, d_tile_item, tiles_per_item, total); break;
    case 6: wbuild_kernel<P, 6, WM><<<grid, block, 0, s>>>(d_items, d_tile_item, tiles_per_item, total); break;
    case 7: wbuild_kernel<P, 7, WM><<<grid, block, 0, s>>>(d_items, d_tile_item, tiles_per_item, total); break;
    case 8: wbuild_kernel<P, 8, WM><<<grid, block, 0, s>>>(d_items, d_tile_item, tiles_per_item, total); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <Prec P>
static hipError_t launch_wb_p(const WItem *d_items, const int *d_tile_item, int tiles_per_item,
                              long total, WConfig c, hipStream_t s) {
  if (c.wm != 2) return hipErrorInvalidValue;  // the only row count instantiated
  return launch_wb_pw<P, 2>(d_items, d_tile_item, tiles_per_item, total, c.nb, s);
}

hipError_t launch_wbuild(Prec p, const WItem *d_items, const int *d_tile_item, int nitems,
                         int tiles_per_item, long total_tiles, WConfig c, hipStream_t s) {
  (void)nitems;
  if (total_tiles <= 0) return hipSuccess;
  if (total_tiles > 0x7fffffffL) return hipErrorInvalidValue;
  switch (p) {
    case Prec::F64: return launch_wb_p<Prec::F64>(d_items, d_tile_item, tiles_per_item, total_tiles, c, s);
    case Prec::F32: return launch_wb_p<Prec::F32>(d_items, d_tile_item, tiles_per_item, total_tiles, c, s);
    case Prec::BF16X3: return launch_wb_p<Prec::BF16X3>(d_items, d_tile_item, tiles_per_item, total_tiles, c, s);
    case Prec::BF16X2: return launch_wb_p<Prec::BF16X2>(d_items, d_tile_item, tiles_per_item, total_tiles, c, s);
    case Prec::FP16X2: return launch_wb_p<Prec::FP16X2>(d_items, d_tile_item, tiles_per_item, total_tiles, c, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace te
