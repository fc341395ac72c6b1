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

// Sixteen zero bytes in global memory: the source of LDS chunks that lie past
// the end of K (the LDS-DMA loads below write whatever their source holds).
__device__ __attribute__((aligned(16))) const unsigned int kZero16[4] = {0u, 0u, 0u, 0u};

typedef __attribute__((address_space(3))) void *lds_ptr;

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

  // two LDS stages as separate objects, so that the compiler can tell the
  // stage being filled by LDS-DMA loads from the one being read
  __shared__ __attribute__((aligned(16))) T As0[NP][BM][LD], As1[NP][BM][LD];
  __shared__ __attribute__((aligned(16))) T Bs0[NP * BN][LD], Bs1[NP * BN][LD];
  using AT = T (*)[BM][LD];
  using BT = T (*)[LD];

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
  const T *TO[2];
  long ksO[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    if (su.om[q] == 0) { TO[q] = reinterpret_cast<const T *>(w.Tr[su.op[q]]); ksO[q] = (long)w.trs; }
    else               { TO[q] = reinterpret_cast<const T *>(w.Tc[su.op[q]]); ksO[q] = (long)w.tcs; }
  }
  // 16-bit modes: occupied-segment rows of the row form (t_{p l}^{yz} with l
  // last, rows of lo); om = 1 takes the swapped pair (t_{l p}^{yz} = t_{p l}^{zy})
  const T *TT0 = reinterpret_cast<const T *>(w.Tt[su.op[0]]);
  const T *TT1 = reinterpret_cast<const T *>(w.Tt[su.op[1]]);

  const int lo = w.lo;
  const int KX = 2 * vp;
  const int KO = TR::SPLIT ? 2 * lo : 2 * o;
  const int nkx = (KX + KT - 1) / KT;
  const int nko = (KO + KT - 1) / KT;
  const int ntiles = nkx + nko;
  constexpr size_t ES = sizeof(T);

  // ---- LDS-DMA loads: the X phase in every precision, and the occupied
  // phase of the 16-bit modes (whose operands are K-contiguous rows too).
  // Wave-load g of a region writes its 16-byte LDS chunks [64 g, 64 g + 64):
  // lane L writes chunk q = 64 g + L, i.e. row q / CR, slot q % CR of the
  // region's part, and so loads the global chunk the swizzle keeps in that
  // slot (slot ^ ((row / RP) % CR)). Rows past the matrix are clamped to row
  // 0 (their products land in rows or columns the epilogue never stores);
  // chunks past the end of K are read from kZero16.
  using SW = Swz<TR>;
  constexpr int EC = SW::EC, CRW = SW::CR, RPW = SW::RP;
  constexpr int GPA = BM * CRW / 64;         // A wave-loads per part
  constexpr int IAP = GPA / 4;               // ... per part and wave
  constexpr int GPB = BN * CRW / 64;         // B wave-loads per part
  constexpr int IB = (NP * GPB + 3) / 4;     // B wave-loads per wave; spare ones
                                             // repeat an earlier block (same bytes)
  static_assert(GPA % 4 == 0, "A tile must split evenly over four waves");
  const int wv = __builtin_amdgcn_readfirstlane(wave);
  uintptr_t pA0[IAP], pA1[IAP];                          // X segment 0 / 1 (minus vp)
  uintptr_t pO0[TR::SPLIT ? IAP : 1], pO1[TR::SPLIT ? IAP : 1];  // row form (minus lo)
  int cA[IAP];                                           // k offset of the chunk
#pragma unroll
  for (int jj = 0; jj < IAP; ++jj) {
    const int q = 64 * (wv * IAP + jj) + lane;
    const int r = q / CRW;
    const int c = (q % CRW) ^ ((r / RPW) % CRW);
    const long m = (long)m0 + r;
    const long mm = m < M ? m : 0;
    const long mx = mm / vp, my = mm - mx * vp;
    cA[jj] = c * EC;
    pA0[jj] = reinterpret_cast<uintptr_t>(XA0) + (uintptr_t)((mm * vp + c * EC) * (long)ES);
    pA1[jj] = reinterpret_cast<uintptr_t>(XA1) + (uintptr_t)(((my * vp + mx) * vp + c * EC - vp) * (long)ES);
    if constexpr (TR::SPLIT) {
      pO0[jj] = reinterpret_cast<uintptr_t>(TT0) +
                (uintptr_t)(((su.om[0] ? my * vp + mx : mm) * lo + c * EC) * (long)ES);
      pO1[jj] = reinterpret_cast<uintptr_t>(TT1) +
                (uintptr_t)(((su.om[1] ? my * vp + mx : mm) * lo + c * EC - lo) * (long)ES);
    }
  }
  // element offsets of the lane's B chunk: in the T2 rows, and (16-bit
  // occupied phase) from the segment's In row base below
  int oB[IB], oI[IB];
  int cB[IB], gB[IB], prB[IB];         // k offset; LDS block and part (uniform)
#pragma unroll
  for (int j = 0; j < IB; ++j) {
    const int g2 = (j * 4 + wv) % (NP * GPB);
    gB[j] = g2;
    prB[j] = g2 / GPB;
    const int q = 64 * (g2 % GPB) + lane;
    const int r = q / CRW;
    const int c = (q % CRW) ^ ((r / RPW) % CRW);
    const int n = n0 + r;
    const long nn = n < vp ? n : 0;
    cB[j] = c * EC;
    oB[j] = (int)(nn * vp + c * EC);
    oI[j] = (int)(nn * o * lo + c * EC);
  }
  // In row (ix, n, iy) starts at ((ix vp + n) o + iy) lo; segment 1's base is
  // taken relative to k = lo
  const T *IB0 = In + ((long)su.ix[0] * vp * o + su.iy[0]) * lo;
  const T *IB1 = In + ((long)su.ix[1] * vp * o + su.iy[1]) * lo - lo;

  auto dma = [](uintptr_t src, char *dst) __attribute__((always_inline)) {
    __builtin_amdgcn_global_load_lds((gptr<u32x4>)src, (lds_ptr)dst, 16, 0, 0);
  };
  const uintptr_t zero = reinterpret_cast<uintptr_t>(kZero16);

  auto issue = [&](int t, AT As, BT Bs) __attribute__((always_inline)) {
    char *sA = reinterpret_cast<char *>(&As[0][0][0]);
    char *sB = reinterpret_cast<char *>(&Bs[0][0]);
    if (t < nkx) {
      const int kb = t * KT;
      if (kb + KT <= vp || (kb >= vp && kb + KT <= KX)) {
        // the whole tile lies in one segment
        const bool s1 = kb >= vp;
        const T *tb = (s1 ? TB1 : TB0) + (kb - (s1 ? vp : 0));
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
          for (int jj = 0; jj < IAP; ++jj)
            dma((s1 ? pA1[jj] : pA0[jj]) + (uintptr_t)(((long)kb + p * (long)w.xps) * (long)ES),
                sA + (p * GPA + wv * IAP + jj) * 1024);
#pragma unroll
        for (int j = 0; j < IB; ++j)
          dma(reinterpret_cast<uintptr_t>(tb + prB[j] * w.tcps + oB[j]), sB + gB[j] * 1024);
      } else {
        // the tile that straddles k = vp, or a ragged last one
#pragma unroll
        for (int p = 0; p < NP; ++p)
#pragma unroll
          for (int jj = 0; jj < IAP; ++jj) {
            const int k = kb + cA[jj];
            const uintptr_t src = (k >= vp ? pA1[jj] : pA0[jj]) +
                                  (uintptr_t)(((long)kb + p * (long)w.xps) * (long)ES);
            dma(k >= KX ? zero : src, sA + (p * GPA + wv * IAP + jj) * 1024);
          }
#pragma unroll
        for (int j = 0; j < IB; ++j) {
          const int k = kb + cB[j];
          const bool s1 = k >= vp;
          const T *tb = (s1 ? TB1 : TB0) + prB[j] * w.tcps + oB[j] + (kb - (s1 ? vp : 0));
          dma(k >= KX ? zero : reinterpret_cast<uintptr_t>(tb), sB + gB[j] * 1024);
        }
      }
    } else if constexpr (TR::SPLIT) {
      const int ko = (t - nkx) * KT;
#pragma unroll
      for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int jj = 0; jj < IAP; ++jj) {
          const int k = ko + cA[jj];
          const uintptr_t src = (k >= lo ? pO1[jj] : pO0[jj]) +
                                (uintptr_t)(((long)ko + p * (long)w.t2tps) * (long)ES);
          dma(k >= KO ? zero : src, sA + (p * GPA + wv * IAP + jj) * 1024);
        }
#pragma unroll
      for (int j = 0; j < IB; ++j) {
        const int k = ko + cB[j];
        const T *ib = (k >= lo ? IB1 : IB0) + prB[j] * w.ips + ko + oI[j];
        dma(k >= KO ? zero : reinterpret_cast<uintptr_t>(ib), sB + gB[j] * 1024);
      }
    }
  };

  // ---- FP64 / FP32 occupied phase: the t2 panels are m-contiguous for a
  // fixed l, so that tile goes through registers and a transposed LDS store.
  // Every load is unconditional, from an address inside its array (a
  // predicated load makes the compiler wait for all loads in flight right
  // away); chunks or elements past K are zeroed when stored.
  constexpr int CA = TR::SPLIT ? 1 : (BM * KT / 8 + WG - 1) / WG;   // 8-element chunks
  constexpr int CB = TR::SPLIT ? 1 : (BN * KT / 8 + WG - 1) / WG;
  constexpr int CPR = KT / 8;
  Chunk<T> ra[CA], rb[CB];
  uint32_t zA[CA], zB[CB];
  long rowI[CB][2];
  int kcB[CB];
#pragma unroll
  for (int u = 0; u < CB; ++u) {
    const int c = tid + u * WG;
    kcB[u] = (c % CPR) * 8;
    const int n = n0 + c / CPR;
    const long nn = (c < BN * CPR && n < vp) ? n : 0;
    rowI[u][0] = (((long)su.ix[0] * vp + nn) * o + su.iy[0]) * lo;
    rowI[u][1] = (((long)su.ix[1] * vp + nn) * o + su.iy[1]) * lo;
  }

  auto load = [&](int t) __attribute__((always_inline)) {
    if constexpr (!TR::SPLIT) {
      // K-major A: thread c takes k = c % KT and eight consecutive m, so the
      // transposed LDS stores of a lane group fill one row (conflict-free)
      const int ko = (t - nkx) * KT;
#pragma unroll
      for (int u = 0; u < CA; ++u) {
        const int c = tid + u * WG;
        const int kg = ko + c % KT;
        const long m = m0 + (c / KT) * 8;
        const bool ok = (c < BM * CPR) && kg < KO && m < M;
        const int seg = ok && kg >= o;
        const long off = ok ? (long)(kg - seg * o) * ksO[seg] + m : 0;
        zA[u] = ok ? 0u : ~0u;
        ra[u].load(TO[seg] + off);
      }
#pragma unroll
      for (int u = 0; u < CB; ++u) {
        uint32_t z = 0;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int kg = ko + kcB[u] + e;
          const bool ok = kg < KO;
          const int seg = ok && kg >= o;
          const long off = rowI[u][seg] + (ok ? kg - seg * o : 0);
          z |= ok ? 0u : 1u << e;
          rb[u].set(e, gld(In + off));
        }
        zB[u] = z;
      }
    }
  };

  auto store = [&](AT As, BT Bs) __attribute__((always_inline)) {
    if constexpr (!TR::SPLIT) {
#pragma unroll
      for (int u = 0; u < CA; ++u) {
        const int c = tid + u * WG;
        if (zA[u]) ra[u].zero();
        if (c < BM * CPR) {
          const int kk = c % KT;
          const int mc = (c / KT) * 8;
#pragma unroll
          for (int e = 0; e < 8; ++e) As[0][mc + e][lcol<TR>(mc + e, kk)] = ra[u].get(e);
        }
      }
#pragma unroll
      for (int u = 0; u < CB; ++u) {
        const int c = tid + u * WG;
#pragma unroll
        for (int e = 0; e < 8; ++e)
          if ((zB[u] >> e) & 1u) rb[u].set(e, T(0));
        if (c < BN * CPR) {
          const int row = c / CPR;
          store_chunk<TR>(&Bs[row][0], row, kcB[u], rb[u]);
        }
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

  // Pipeline: two LDS stages; the next tile's loads are in flight while this
  // one is computed. The barrier is the bare s_barrier after an explicit
  // wait for this wave's loads and LDS accesses (a __syncthreads fence would
  // also order the LDS-DMA writes against every later LDS read and make the
  // compiler wait for the next tile's loads before computing this one).
  auto sync = [] {
    __builtin_amdgcn_sched_barrier(0);   // the tile's MFMAs issue before the wait
    __builtin_amdgcn_s_waitcnt(0);       // vmcnt(0) expcnt(0) lgkmcnt(0)
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_sched_barrier(0);
  };
  auto compute = [&](AT As, BT Bs) __attribute__((always_inline)) {
#pragma unroll
    for (int kk = 0; kk < KT / KM; ++kk) {
      if constexpr (NP == 1) {
        using E = T;
        E av[WM], bv[NB];
#pragma unroll
        for (int rb_ = 0; rb_ < WM; ++rb_) {
          const int r = wrow + rb_ * 16 + fr;
          av[rb_] = As[0][r][lcol<TR>(r, kk * 4 + fk)];
        }
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) bv[cb] = Bs[cb * 16 + fr][lcol<TR>(cb * 16 + fr, kk * 4 + fk)];
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
                &As[p][wrow + rb_ * 16 + fr][lcol<TR>(wrow + rb_ * 16 + fr, fk * 8)]);
#pragma unroll
        for (int cb = 0; cb < NB; ++cb)
#pragma unroll
          for (int p = 0; p < NP; ++p)
            bv[cb][p] = *reinterpret_cast<const F *>(&Bs[p * BN + cb * 16 + fr][lcol<TR>(cb * 16 + fr, fk * 8)]);
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
  };

  // LDS-DMA tiles: every tile in the 16-bit modes, the X phase otherwise.
  // The loop runs two tiles per trip so that each stage is a fixed object;
  // the loads are issued unconditionally (past the last tile they fetch it
  // again into the stage no longer read), which keeps the compiler's wait
  // accounting exact.
  const int ndma = TR::SPLIT ? ntiles : nkx;
  auto dma_step = [&](int t, AT Ac, BT Bc, AT An, BT Bn) __attribute__((always_inline)) {
    issue(t + 1 < ndma ? t + 1 : ndma - 1, An, Bn);
    compute(Ac, Bc);
    sync();
  };
  issue(0, As0, Bs0);
  sync();
  int t = 0;
  for (; t + 1 < ndma; t += 2) {
    dma_step(t, As0, Bs0, As1, Bs1);
    dma_step(t + 1, As1, Bs1, As0, Bs0);
  }
  if (t < ndma) {
    dma_step(t, As0, Bs0, As1, Bs1);
    ++t;
  }
  // FP64 / FP32 occupied phase through registers (stages continue to
  // alternate; t is the next tile)
  if constexpr (!TR::SPLIT) {
    if (t < ntiles) {
      const bool odd = t & 1;
      load(t);
      store(odd ? AT(As1) : AT(As0), odd ? BT(Bs1) : BT(Bs0));
      sync();
      for (; t < ntiles; ++t) {
        const bool cur1 = t & 1;
        if (t + 1 < ntiles) load(t + 1);
        compute(cur1 ? AT(As1) : AT(As0), cur1 ? BT(Bs1) : BT(Bs0));
        if (t + 1 < ntiles) store(cur1 ? AT(As0) : AT(As1), cur1 ? BT(Bs0) : BT(Bs1));
        sync();
      }
    }
  }

  // epilogue: boxed store of this GEMM's share of W, with one division per
  // output row. Store order: row by row for FP64 (ROWQ = 1); for the FP32
  // outputs a 16 x 16 block at a time (four stores cover it: rows 4 (l / 16)
  // + r), which measured 5-10% faster there than row by row.
  Out *Wg = reinterpret_cast<Out *>(w.W) + (long)g * vp2 * vp;
  const int nT = vp >> 3;
  auto put = [&](int rb_, int cb, int r, long m, int p0, int p1) __attribute__((always_inline)) {
    const int n = n0 + cb * 16 + fr;
    if (m < M && n < vp) {
      int a, b, c;
      if (g == 0) { a = p0; b = p1; c = n; }
      else if (g == 1) { a = n; b = p0; c = p1; }
      else { a = p0; b = n; c = p1; }
      Out x = (Out)acc[rb_][cb][r];
      if constexpr (TR::SCALED) x *= w.scale;
      gst(Wg + box_off(a, b, c, nT), x);
    }
  };
#pragma unroll
  for (int rb_ = 0; rb_ < WM; ++rb_) {
    long m[4];
    int p0[4], p1[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      m[r] = m0 + wrow + rb_ * 16 + (TR::ROWQ == 1 ? fk + 4 * r : fk * 4 + r);
      p0[r] = (int)(m[r] / vp);
      p1[r] = (int)(m[r] - (long)p0[r] * vp);
    }
    if constexpr (TR::ROWQ == 1) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) put(rb_, cb, r, m[r], p0[r], p1[r]);
    } else {
#pragma unroll
      for (int cb = 0; cb < NB; ++cb)
#pragma unroll
        for (int r = 0; r < 4; ++r) put(rb_, cb, r, m[r], p0[r], p1[r]);
    }
  }
}

}  // namespace

// ------------------------------------------------------------ launchers
// Tile shape: two 16-row blocks per wave in every precision, and the
// column-block count NB in [4, 8] that minimises padded waste of the lone
// index (larger NB on ties). (Wide tiles at one workgroup per CU, 256 x 208
// or 128 x 400, load half the operand bytes per MFMA but ran the 16-bit and
// FP32 W builds 3-19% slower than three 128 x 80 workgroups per CU.)
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
