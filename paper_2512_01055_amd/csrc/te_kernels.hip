// gfx950 kernels of the (T) library.
//
//  wbuild_kernel   W^{abc}_{ijk} of Eq. 2 summed over the pair permutations of
//                  Eq. 5, as three MFMA GEMMs per occupied triple (one per
//                  virtual index that stands alone in a term).
//  energy_kernel   V (Eq. 3), D (Eq. 4, sign of the energy-kernel figure), the
//                  permutation combination Z and (W + V) Z / D of Eq. 1, over
//                  one sextet of 8^3 W boxes per workgroup.
//  reduce/sum      fixed-order FP64 reductions (bitwise reproducible).
//  gemm_tn         FP64 MFMA product used to assemble integrals from the
//                  factors (Eq. 6) at staging.
//  conversions     FP64 -> FP32 and FP64 -> split BF16 operand copies.
#include "te_internal.h"

#include <stdint.h>

namespace te {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int WG = 256;

// ---------------------------------------------------------------- traits
template <Prec P> struct Tr;
// Output lane layout of the 16x16 MFMA blocks: lane l, register r holds
// column l%16 and row  (l/16) + 4r  for v_mfma_f64_16x16x4f64  (ROWQ = 1),
//                      4(l/16) + r  for the FP32 and BF16 forms (ROWQ = 4).
//
// LDS tiles are unpadded rows of KT elements. The 16-byte chunks of a row are
// XOR-swizzled: chunk c of row r is stored at chunk c ^ ((r / RP) % CR), with
// RP rows per 256 bytes (64 banks) and CR chunks per row. The 16 rows one
// fragment read touches then fall in 16 distinct bank groups, and no padding
// is spent, which is what lets two (BF16x3, FP64) or three (FP32, BF16x2)
// workgroups share a CU.
template <> struct Tr<Prec::F64> {
  using T = double; using Acc = d4; using Out = double;
  static constexpr int KT = 16, PAD = 0, NP = 1, KM = 4, ROWQ = 1;
  static constexpr bool SPLIT = false;
};
template <> struct Tr<Prec::F32> {
  using T = float; using Acc = f4; using Out = float;
  static constexpr int KT = 32, PAD = 0, NP = 1, KM = 4, ROWQ = 4;
  static constexpr bool SPLIT = false;
};
template <> struct Tr<Prec::BF16X3> {
  using T = uint16_t; using Acc = f4; using Out = float;
  static constexpr int KT = 32, PAD = 0, NP = 3, KM = 32, ROWQ = 4;
  static constexpr bool SPLIT = true;
};
template <> struct Tr<Prec::BF16X2> {
  using T = uint16_t; using Acc = f4; using Out = float;
  static constexpr int KT = 32, PAD = 0, NP = 2, KM = 32, ROWQ = 4;
  static constexpr bool SPLIT = true;
};

template <typename TR> struct Swz {
  static constexpr int EC = 16 / sizeof(typename TR::T);            // elements per chunk
  static constexpr int CR = TR::KT / EC;                             // chunks per row
  static constexpr int RP = 256 / (TR::KT * (int)sizeof(typename TR::T));  // rows per 256 B
};
// Column of element k of LDS row r.
template <typename TR> __device__ inline int lcol(int r, int k) {
  using S = Swz<TR>;
  return ((((k / S::EC) ^ ((r / S::RP) % S::CR))) * S::EC) | (k % S::EC);
}
// Store eight consecutive elements (k0 % 8 == 0) of row r as swizzled chunks.
template <typename TR, typename T, typename CH>
__device__ inline void store_chunk(T *row, int r, int k0, const CH &c) {
  using S = Swz<TR>;
#pragma unroll
  for (int q = 0; q < CH::NQ; ++q)
    *reinterpret_cast<u32x4 *>(row + lcol<TR>(r, k0 + q * S::EC)) = c.q[q];
}

// Global-address-space views. Operand pointers reach the kernels through
// item structs in memory, so the compiler sees generic pointers and would
// emit FLAT accesses; FLAT loads count against the LDS counter too, which
// makes every wait for LDS fragments also wait for the next tile's prefetch.
template <typename T> using gptr = const __attribute__((address_space(1))) T *;
template <typename T> using gptr_w = __attribute__((address_space(1))) T *;
template <typename T> __device__ inline T gld(const T *p) { return *(gptr<T>)(p); }
template <typename T> __device__ inline void gst(T *p, T x) { *(gptr_w<T>)(p) = x; }

// Eight consecutive elements, moved as 16-byte words.
template <typename T> struct Chunk {
  static constexpr int NQ = sizeof(T) * 8 / 16;
  u32x4 q[NQ];
  __device__ T get(int e) const { return reinterpret_cast<const T *>(q)[e]; }
  __device__ void set(int e, T x) { reinterpret_cast<T *>(q)[e] = x; }
  __device__ void zero() {
#pragma unroll
    for (int i = 0; i < NQ; ++i) q[i] = u32x4{0u, 0u, 0u, 0u};
  }
  __device__ void load(const T *p) {
    gptr<u32x4> s = (gptr<u32x4>)(p);
#pragma unroll
    for (int i = 0; i < NQ; ++i) q[i] = s[i];
  }
};

__device__ inline d4 mma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4 mma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline f4 mma(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ inline long box_off(int a, int b, int c, int nT) {
  return ((((long)(a >> 3) * nT + (b >> 3)) * nT + (c >> 3)) << 9) + ((a & 7) << 6) +
         ((b & 7) << 3) + (c & 7);
}

// Logical tile id such that consecutive ids share an XCD (workgroups are
// dispatched round-robin over the 8 XCDs of the chip).
__device__ inline long xcd_remap(long bid, long total) {
  long per = total >> 3, rem = total & 7;
  long x = bid & 7, q = bid >> 3;
  return x * per + (x < rem ? x : rem) + q;
}

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
struct Setup {
  int xa[2];      // X slice (0: X_i, 1: X_j, 2: X_k) of segments 0/1 (seg 1 transposed)
  int tq[2], tr[2];  // T_{tq tr} rows for the B side of segments 0/1
  int op[2], om[2];  // occupied-term A side: om 0 -> t2[op][l], 1 -> t2[l][op]
  int ix[2], iy[2];  // In_{ix iy} rows for segments 2/3
};

__device__ inline Setup make_setup(int g, int i, int j, int k) {
  Setup s;
  if (g == 0) {
    s.xa[0] = 0; s.xa[1] = 1;
    s.tq[0] = k; s.tr[0] = j; s.tq[1] = k; s.tr[1] = i;
    s.op[0] = i; s.om[0] = 0; s.op[1] = j; s.om[1] = 1;
    s.ix[0] = k; s.iy[0] = j; s.ix[1] = k; s.iy[1] = i;
  } else if (g == 1) {
    s.xa[0] = 1; s.xa[1] = 2;
    s.tq[0] = i; s.tr[0] = k; s.tq[1] = i; s.tr[1] = j;
    s.op[0] = k; s.om[0] = 1; s.op[1] = j; s.om[1] = 0;
    s.ix[0] = i; s.iy[0] = j; s.ix[1] = i; s.iy[1] = k;
  } else {
    s.xa[0] = 0; s.xa[1] = 2;
    s.tq[0] = j; s.tr[0] = k; s.tq[1] = j; s.tr[1] = i;
    s.op[0] = k; s.om[0] = 1; s.op[1] = i; s.om[1] = 0;
    s.ix[0] = j; s.iy[0] = i; s.ix[1] = j; s.iy[1] = k;
  }
  return s;
}

// NB: 16-column blocks per tile (BN = 16 NB); WM: 16-row blocks per wave
// (BM = 4 waves x 16 WM rows). The register budget asks for three waves per
// SIMD; that is what the two-part BF16 tiles' LDS allows (the other modes are
// held to two by LDS and are not constrained by it).
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
  constexpr int CAO = BM / 8;                     // O-phase A: chunks per k row

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
  const T *T2 = reinterpret_cast<const T *>(w.T2);
  const T *In = reinterpret_cast<const T *>(w.In);

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
  long rowB[CB][2];
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
    rowB[u][0] = (((long)su.tq[0] * o + su.tr[0]) * vp + nn) * vp;
    rowB[u][1] = (((long)su.tq[1] * o + su.tr[1]) * vp + nn) * vp;
  }
  long baseO[2], ksO[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    if (su.om[s] == 0) { baseO[s] = (long)su.op[s] * o * vp2; ksO[s] = vp2; }
    else               { baseO[s] = (long)su.op[s] * vp2;     ksO[s] = (long)o * vp2; }
  }
  // BF16 modes: occupied-segment rows of T2T (t_{p l}^{yz} with l last), read
  // like the X rows; om = 1 takes the swapped pair (t_{l p}^{yz} = t_{p l}^{zy})
  const int lo = w.lo;
  const T *T2T = reinterpret_cast<const T *>(w.T2T);
  long rowO[TR::SPLIT ? CA : 1][2];
  if constexpr (TR::SPLIT) {
#pragma unroll
    for (int u = 0; u < CA; ++u) {
      long mm = okA[u] ? (long)m0 + (tid + u * WG) / CPR : 0;
      long mx = mm / vp, my = mm - mx * vp;
#pragma unroll
      for (int s = 0; s < 2; ++s)
        rowO[u][s] = ((long)su.op[s] * vp2 + (su.om[s] ? my * vp + mx : mm)) * lo;
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
        long off = rowB[u][seg] + (kg - seg * vp);
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          if (ok) rb[u][p].load(T2 + p * w.tps + off); else rb[u][p].zero();
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
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          if (ok) ra[u][p].load(T2T + p * w.t2tps + off); else ra[u][p].zero();
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
      const int kb = (t - nkx) * KT;
#pragma unroll
      for (int u = 0; u < CA; ++u) {
        int c = tid + u * WG;
        int kk = c / CAO;
        int mc = (c % CAO) * 8;
        int kg = kb + kk;
        long m = m0 + mc;
        bool ok = (c < BM * CPR) && kg < KO && m < M;
        int seg = kg >= o;
        long off = baseO[seg] + (long)(kg - seg * o) * ksO[seg] + m;
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          if (ok) ra[u][p].load(T2 + p * w.tps + off); else ra[u][p].zero();
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
          int kk = c / CAO;
          int mc = (c % CAO) * 8;
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
        bf8 av[WM][NP], bv[NB][NP];
#pragma unroll
        for (int rb_ = 0; rb_ < WM; ++rb_)
#pragma unroll
          for (int p = 0; p < NP; ++p)
            av[rb_][p] = *reinterpret_cast<const bf8 *>(
                &As[cur][p][wrow + rb_ * 16 + fr][lcol<TR>(wrow + rb_ * 16 + fr, fk * 8)]);
#pragma unroll
        for (int cb = 0; cb < NB; ++cb)
#pragma unroll
          for (int p = 0; p < NP; ++p)
            bv[cb][p] = *reinterpret_cast<const bf8 *>(&Bs[cur][p][cb * 16 + fr][lcol<TR>(cb * 16 + fr, fk * 8)]);
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
          gst(Wg + box_off(a, b, c, nT), (Out)acc[rb_][cb][r]);
        }
      }
}

// ------------------------------------------------------------ energy
//
// Slot s of the sextet holds box (T[P_s[0]], T[P_s[1]], T[P_s[2]]) with
// (T[0], T[1], T[2]) = (A, B, C), A >= B >= C. An element at local (x0,x1,x2)
// of slot s permuted by q sits in slot PERM_COMP[s][q] at (x_q0, x_q1, x_q2).
__constant__ int c_perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 1, 0}, {2, 0, 1}};
__constant__ int c_comp[6][6] = {
    // comp[s][q] = index of (P_s[P_q[0]], P_s[P_q[1]], P_s[P_q[2]])
    {0, 1, 2, 3, 4, 5}, {1, 0, 5, 4, 3, 2}, {2, 3, 0, 1, 5, 4},
    {3, 2, 4, 5, 1, 0}, {4, 5, 3, 2, 0, 1}, {5, 4, 1, 0, 2, 3}};

constexpr int BX_R = 9;             // padded row   (x2 stride 1, x1 stride 9)
constexpr int BX_P = 8 * BX_R + 1;  // padded plane (x0 stride 73)
constexpr int BX_S = 8 * BX_P;      // slot size in doubles

__device__ inline int bxi(int x0, int x1, int x2) { return x0 * BX_P + x1 * BX_R + x2; }

template <typename WT>
__global__ __launch_bounds__(WG) void energy_kernel(const EItem *__restrict__ items,
                                                    const int *__restrict__ blk_item,
                                                    int blks_per_item, long total) {
  __shared__ double box[6 * BX_S];
  __shared__ double red[WG / 64];
  const int tid = threadIdx.x;
  const long bid = blockIdx.x;
  int it;
  long local;
  if (blk_item) {
    it = blk_item[bid];
    local = bid - blk_item[total + it];
  } else {
    it = (int)(bid / blks_per_item);
    local = bid - (long)it * blks_per_item;
  }
  const EItem &e = items[it];
  const int o = e.o, v = e.v, vp = e.vp, nT = e.nT;
  const int i = e.i, j = e.j, k = e.k;
  const int packed = e.sext[local];
  int T[3] = {packed & 1023, (packed >> 10) & 1023, (packed >> 20) & 1023};

  int bx[6][3];
  int canon[6];
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    bx[s][0] = T[c_perm[s][0]]; bx[s][1] = T[c_perm[s][1]]; bx[s][2] = T[c_perm[s][2]];
    canon[s] = s;
    for (int q = 0; q < s; ++q)
      if (canon[s] == s && bx[q][0] == bx[s][0] && bx[q][1] == bx[s][1] && bx[q][2] == bx[s][2])
        canon[s] = q;
  }

  const long vp3 = (long)vp * vp * vp;
  const WT *W0 = reinterpret_cast<const WT *>(e.W);
  const WT *W1 = W0 + vp3;
  const WT *W2 = W1 + vp3;
  for (int idx = tid; idx < 6 * BOX3; idx += WG) {
    int s = idx >> 9;
    if (canon[s] != s) continue;
    int r = idx & (BOX3 - 1);
    long base = ((((long)bx[s][0] * nT + bx[s][1]) * nT + bx[s][2]) << 9) + r;
    double wv = ((double)gld(W0 + base) + (double)gld(W1 + base)) + (double)gld(W2 + base);
    box[s * BX_S + bxi(r >> 6, (r >> 3) & 7, r & 7)] = wv;
  }
  __syncthreads();

  const double eijk = (e.eo[i] + e.eo[j]) + e.eo[k];
  const double *t1i = e.t1 + (long)i * vp, *t1j = e.t1 + (long)j * vp, *t1k = e.t1 + (long)k * vp;
  double acc = 0.0;
#pragma unroll 1
  for (int s = 0; s < 6; ++s) {
    if (canon[s] != s) continue;
    const int sb = canon[c_comp[s][3]] * BX_S;  // (b,c,a)
    const int sc = canon[c_comp[s][5]] * BX_S;  // (c,a,b)
    const int sd = canon[c_comp[s][1]] * BX_S;  // (a,c,b)
    const int se = canon[c_comp[s][2]] * BX_S;  // (b,a,c)
    const int sf = canon[c_comp[s][4]] * BX_S;  // (c,b,a)
    for (int r = tid; r < BOX3; r += WG) {
      const int x0 = r >> 6, x1 = (r >> 3) & 7, x2 = r & 7;
      const int a = bx[s][0] * 8 + x0, b = bx[s][1] * 8 + x1, c = bx[s][2] * 8 + x2;
      if (a < v && b < v && c < v) {
        const double w0 = box[s * BX_S + bxi(x0, x1, x2)];
        const double z = 4.0 * w0 + box[sb + bxi(x1, x2, x0)] + box[sc + bxi(x2, x0, x1)]
                         - 2.0 * box[sd + bxi(x0, x2, x1)] - 2.0 * box[se + bxi(x1, x0, x2)]
                         - 2.0 * box[sf + bxi(x2, x1, x0)];
        // singles term (Eq. 3): t_i^a (jb|kc) + t_j^b (ia|kc) + t_k^c (ia|jb)
        const double vt = gld(t1i + a) * gld(e.K + (((long)j * vp + b) * o + k) * vp + c)
                        + gld(t1j + b) * gld(e.K + (((long)i * vp + a) * o + k) * vp + c)
                        + gld(t1k + c) * gld(e.K + (((long)i * vp + a) * o + j) * vp + b);
        const double d = ((eijk - gld(e.ev + a)) - gld(e.ev + b)) - gld(e.ev + c);
        acc += (w0 + vt) * z / d;
      }
    }
  }
  // fixed-order reduction: butterfly within the wave, then waves in order
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((tid & 63) == 0) red[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) {
    double sum = red[0];
#pragma unroll
    for (int q = 1; q < WG / 64; ++q) sum += red[q];
    e.part[local] = sum;
  }
}

// ------------------------------------------------------------ reductions
__device__ inline double block_sum(double x, double *red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
  const int tid = threadIdx.x;
  if ((tid & 63) == 0) red[tid >> 6] = x;
  __syncthreads();
  double s = 0.0;
  if (tid == 0) {
    s = red[0];
    for (int q = 1; q < (int)(blockDim.x >> 6); ++q) s += red[q];
  }
  return s;
}

__global__ __launch_bounds__(WG) void reduce_kernel(const RItem *__restrict__ items) {
  __shared__ double red[WG / 64];
  const RItem r = items[blockIdx.x];
  double x = 0.0;
  for (int q = threadIdx.x; q < r.n; q += WG) x += r.part[q];
  double s = block_sum(x, red);
  if (threadIdx.x == 0) *r.out = r.w * s;
}

__global__ __launch_bounds__(1024) void sum_kernel(const double *__restrict__ x, long n,
                                                   double *out) {
  __shared__ double red[1024 / 64];
  double a = 0.0;
  for (long q = threadIdx.x; q < n; q += 1024) a += x[q];
  double s = block_sum(a, red);
  if (threadIdx.x == 0) *out = s;
}

// ------------------------------------------------------------ staging GEMM
constexpr int GT = 64, GK = 16;

__global__ __launch_bounds__(WG) void gemm_tn_kernel(GemmTN g) {
  __shared__ double As[GK][GT];
  __shared__ double Bs[GK][GT];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.x * GT, n0 = blockIdx.y * GT;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  d4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int r = 0; r < 4; ++r) acc[a][b][r] = 0.0;
  for (int k0 = 0; k0 < g.K; k0 += GK) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      int e = tid * 4 + u;
      int q = e / GT, c = e % GT;
      int kq = k0 + q;
      As[q][c] = (kq < g.K && m0 + c < g.M) ? g.A[(long)kq * g.lda + m0 + c] : 0.0;
      Bs[q][c] = (kq < g.K && n0 + c < g.N) ? g.B[(long)kq * g.ldb + n0 + c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; kk += 4) {
      double av[2], bv[2];
      for (int a = 0; a < 2; ++a) av[a] = As[kk + (lane >> 4)][wm + a * 16 + (lane & 15)];
      for (int b = 0; b < 2; ++b) bv[b] = Bs[kk + (lane >> 4)][wn + b * 16 + (lane & 15)];
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) acc[a][b] = mma(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int r = 0; r < 4; ++r) {
        int m = m0 + wm + a * 16 + (lane >> 4) + 4 * r;   // FP64 MFMA row order
        int n = n0 + wn + b * 16 + (lane & 15);
        if (m < g.M && n < g.N) {
          long ro = (long)(m / g.rd) * g.rs1 + (long)(m % g.rd) * g.rs2;
          long co = (long)(n / g.cd) * g.cs1 + (long)(n % g.cd) * g.cs2;
          g.C[ro + co] = g.alpha * acc[a][b][r];
        }
      }
}

// ------------------------------------------------------------ element-wise
__global__ void pad4_kernel(const double *__restrict__ src, double *__restrict__ dst, int d0,
                            int d1, int d2, int d3, int p1, int p2, int p3, double scale) {
  long n = (long)d0 * d1 * d2 * d3;
  for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n;
       q += (long)gridDim.x * blockDim.x) {
    long r = q;
    int x3 = r % d3; r /= d3;
    int x2 = r % d2; r /= d2;
    int x1 = r % d1; r /= d1;
    int x0 = (int)r;
    dst[(((long)x0 * p1 + x1) * p2 + x2) * p3 + x3] = scale * src[q];
  }
}

__global__ void to_f32_kernel(const double *__restrict__ src, float *__restrict__ dst, size_t n) {
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n;
       q += (size_t)gridDim.x * blockDim.x)
    dst[q] = (float)src[q];
}

__device__ inline uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline double bf16_val(uint16_t h) {
  return (double)__uint_as_float(((uint32_t)h) << 16);
}

// x ~ sum_p h_p, h_p = bf16(x - sum_{q<p} h_q); parts stored [part][n]
__global__ void to_bf16_parts_kernel(const double *__restrict__ src, uint16_t *__restrict__ dst,
                                     size_t n, int nparts) {
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n;
       q += (size_t)gridDim.x * blockDim.x) {
    double r = src[q];
    for (int p = 0; p < nparts; ++p) {
      uint16_t h = bf16_rne((float)r);
      dst[p * n + q] = h;
      r -= bf16_val(h);
    }
  }
}

__device__ inline void split_store(double r, uint16_t *dst, size_t q, size_t n, int nparts) {
  for (int p = 0; p < nparts; ++p) {
    uint16_t h = bf16_rne((float)r);
    dst[p * n + q] = h;
    r -= bf16_val(h);
  }
}

__global__ void t2t_bf16_kernel(const double *__restrict__ t2, uint16_t *__restrict__ dst, int o,
                                int vp, int lo, int nparts) {
  const long vp2 = (long)vp * vp;
  const size_t n = (size_t)o * vp2 * lo;
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n;
       q += (size_t)gridDim.x * blockDim.x) {
    const int l = (int)(q % lo);
    const size_t r = q / lo;
    const long pair = (long)(r % vp2);
    const int p = (int)(r / vp2);
    const double x = l < o ? t2[((long)p * o + l) * vp2 + pair] : 0.0;
    split_store(x, dst, q, n, nparts);
  }
}

__global__ void in_bf16_kernel(const double *__restrict__ in, uint16_t *__restrict__ dst, int o,
                               int vp, int lo, int nparts) {
  const size_t n = (size_t)o * vp * o * lo;
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n;
       q += (size_t)gridDim.x * blockDim.x) {
    const int l = (int)(q % lo);
    const size_t r = q / lo;                  // (p, x, q') row
    const double x = l < o ? in[r * o + l] : 0.0;
    split_store(x, dst, q, n, nparts);
  }
}

__global__ void check_kernel(const double *__restrict__ x, size_t n, int *flag) {
  int bad = 0;
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n;
       q += (size_t)gridDim.x * blockDim.x)
    bad |= !isfinite(x[q]);
  if (bad) atomicOr(flag, 1);
}

// max |t2[i][j][a][b] - t2[j][i][b][a]| and max |t2| via bit patterns of
// non-negative doubles (ordered like the values)
__global__ void t2_asym_kernel(const double *__restrict__ t2, int o, int v,
                               unsigned long long *out) {
  long n = (long)o * o * v * v;
  double md = 0.0, ma = 0.0;
  for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < n;
       q += (long)gridDim.x * blockDim.x) {
    long r = q;
    int b = r % v; r /= v;
    int a = r % v; r /= v;
    int j = r % o; r /= o;
    int i = (int)r;
    double x = t2[q];
    double y = t2[(((long)j * o + i) * v + b) * v + a];
    md = fmax(md, fabs(x - y));
    ma = fmax(ma, fabs(x));
  }
  atomicMax(&out[0], (unsigned long long)__double_as_longlong(md));
  atomicMax(&out[1], (unsigned long long)__double_as_longlong(ma));
}

// ------------------------------------------------------------ MFMA rate probe
// Eight independent accumulator chains per wave, operands in registers: the
// matrix pipe never waits for memory. The result is written so the chains
// are not optimised away.
template <typename V, typename A, int NCH>
__device__ inline void mfma_chains(V x, V y, A *acc, int iters) {
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int c = 0; c < NCH; ++c) acc[c] = mma(x, y, acc[c]);
}

__global__ __launch_bounds__(WG) void probe_f64(double *out, int iters) {
  d4 acc[8];
  for (int c = 0; c < 8; ++c) acc[c] = d4{0, 0, 0, 0};
  const double x = 1.0 + 1e-9 * threadIdx.x, y = 1.0 - 1e-9 * threadIdx.x;
  mfma_chains<double, d4, 8>(x, y, acc, iters);
  double s = 0;
  for (int c = 0; c < 8; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  gst(out + blockIdx.x * (long)WG + threadIdx.x, s);
}

__global__ __launch_bounds__(WG) void probe_f32(float *out, int iters) {
  f4 acc[8];
  for (int c = 0; c < 8; ++c) acc[c] = f4{0, 0, 0, 0};
  const float x = 1.0f + 1e-6f * threadIdx.x, y = 1.0f;
  mfma_chains<float, f4, 8>(x, y, acc, iters);
  float s = 0;
  for (int c = 0; c < 8; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  gst(out + blockIdx.x * (long)WG + threadIdx.x, s);
}

__global__ __launch_bounds__(WG) void probe_bf16(float *out, int iters) {
  f4 acc[8];
  for (int c = 0; c < 8; ++c) acc[c] = f4{0, 0, 0, 0};
  bf8 x, y;
  for (int e = 0; e < 8; ++e) {
    x[e] = (__bf16)(float)((threadIdx.x + e) & 7);
    y[e] = (__bf16)(float)(e - 3);
  }
  mfma_chains<bf8, f4, 8>(x, y, acc, iters);
  float s = 0;
  for (int c = 0; c < 8; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  gst(out + blockIdx.x * (long)WG + threadIdx.x, s);
}

}  // namespace

// flops of one probe launch: blocks x 4 waves x 8 chains x iters x MFMA flops
hipError_t launch_mfma_probe(Prec p, void *out, int blocks, int iters, hipStream_t s,
                             double *flops) {
  const double per = p == Prec::F64 ? 2.0 * 16 * 16 * 4 : (p == Prec::F32 ? 2.0 * 16 * 16 * 4
                                                                           : 2.0 * 16 * 16 * 32);
  *flops = per * 8.0 * iters * blocks * (WG / 64);
  if (p == Prec::F64) probe_f64<<<blocks, WG, 0, s>>>((double *)out, iters);
  else if (p == Prec::F32) probe_f32<<<blocks, WG, 0, s>>>((float *)out, iters);
  else probe_bf16<<<blocks, WG, 0, s>>>((float *)out, iters);
  return hipGetLastError();
}

// ------------------------------------------------------------ launchers
// Tile shape per precision: rows per wave (WM) and the column-block count
// NB in [4, 8] that minimises padded waste of the lone index (larger NB on
// ties).
WConfig wbuild_config(Prec p, int vp) {
  WConfig c;
  c.wm = (p == Prec::F64) ? 2 : 2;
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
  if (c.wm == 2) return launch_wb_pw<P, 2>(d_items, d_tile_item, tiles_per_item, total, c.nb, s);
  if constexpr (P != Prec::BF16X3) {  // three BF16 parts of a 256-row tile exceed LDS
    if (c.wm == 4) return launch_wb_pw<P, 4>(d_items, d_tile_item, tiles_per_item, total, c.nb, s);
  }
  return hipErrorInvalidValue;
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
  }
  return hipErrorInvalidValue;
}

hipError_t launch_energy(bool w_is_f64, const EItem *d_items, const int *d_blk_item, int nitems,
                         int blks_per_item, long total_blks, hipStream_t s) {
  (void)nitems;
  if (total_blks <= 0) return hipSuccess;
  if (total_blks > 0x7fffffffL) return hipErrorInvalidValue;
  dim3 grid((unsigned)total_blks), block(WG);
  if (w_is_f64)
    energy_kernel<double><<<grid, block, 0, s>>>(d_items, d_blk_item, blks_per_item, total_blks);
  else
    energy_kernel<float><<<grid, block, 0, s>>>(d_items, d_blk_item, blks_per_item, total_blks);
  return hipGetLastError();
}

hipError_t launch_reduce(const RItem *d_items, int nitems, hipStream_t s) {
  if (nitems <= 0) return hipSuccess;
  reduce_kernel<<<dim3(nitems), dim3(WG), 0, s>>>(d_items);
  return hipGetLastError();
}

hipError_t launch_sum(const double *x, long n, double *out, hipStream_t s) {
  sum_kernel<<<dim3(1), dim3(1024), 0, s>>>(x, n, out);
  return hipGetLastError();
}

hipError_t launch_gemm_tn(const GemmTN &g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  dim3 grid((g.M + GT - 1) / GT, (g.N + GT - 1) / GT);
  if (grid.y > 65535) return hipErrorInvalidValue;
  gemm_tn_kernel<<<grid, dim3(WG), 0, s>>>(g);
  return hipGetLastError();
}

static unsigned blocks_for(size_t n) {
  size_t b = (n + WG - 1) / WG;
  return (unsigned)(b > 65536 ? 65536 : (b == 0 ? 1 : b));
}

hipError_t launch_pad4(const double *src, double *dst, int d0, int d1, int d2, int d3, int p1,
                       int p2, int p3, double scale, hipStream_t s) {
  size_t n = (size_t)d0 * d1 * d2 * d3;
  pad4_kernel<<<blocks_for(n), WG, 0, s>>>(src, dst, d0, d1, d2, d3, p1, p2, p3, scale);
  return hipGetLastError();
}

hipError_t launch_to_f32(const double *src, float *dst, size_t n, hipStream_t s) {
  to_f32_kernel<<<blocks_for(n), WG, 0, s>>>(src, dst, n);
  return hipGetLastError();
}

hipError_t launch_to_bf16_parts(const double *src, uint16_t *dst, size_t n, int nparts,
                                hipStream_t s) {
  to_bf16_parts_kernel<<<blocks_for(n), WG, 0, s>>>(src, dst, n, nparts);
  return hipGetLastError();
}

hipError_t launch_t2t_bf16_parts(const double *t2, uint16_t *dst, int o, int vp, int lo,
                                 int nparts, hipStream_t s) {
  size_t n = (size_t)o * vp * vp * lo;
  t2t_bf16_kernel<<<blocks_for(n), WG, 0, s>>>(t2, dst, o, vp, lo, nparts);
  return hipGetLastError();
}

hipError_t launch_in_bf16_parts(const double *in, uint16_t *dst, int o, int vp, int lo,
                                int nparts, hipStream_t s) {
  size_t n = (size_t)o * vp * o * lo;
  in_bf16_kernel<<<blocks_for(n), WG, 0, s>>>(in, dst, o, vp, lo, nparts);
  return hipGetLastError();
}

hipError_t launch_check(const double *x, size_t n, int *flag, hipStream_t s) {
  check_kernel<<<blocks_for(n), WG, 0, s>>>(x, n, flag);
  return hipGetLastError();
}

hipError_t launch_t2_asym(const double *t2, int o, int v, double *out2, double *unused,
                          hipStream_t s) {
  (void)unused;
  size_t n = (size_t)o * o * v * v;
  t2_asym_kernel<<<blocks_for(n), WG, 0, s>>>(t2, o, v,
                                               reinterpret_cast<unsigned long long *>(out2));
  return hipGetLastError();
}

}  // namespace te
