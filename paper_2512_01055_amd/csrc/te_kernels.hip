// gfx950 kernels of the (T) library other than the W build.
//
//  energy_kernel   V (Eq. 3), D (Eq. 4, sign of the energy-kernel figure), the
//                  permutation combination Z and (W + V) Z / D of Eq. 1, over
//                  sextets of 8^3 W boxes (up to eight per workgroup, the next
//                  one's loads in flight while one is evaluated).
//  reduce/sum      fixed-order FP64 reductions (bitwise reproducible).
//  gemm_tn         FP64 MFMA product used to assemble integrals from the
//                  factors (Eq. 6) at staging.
//  conversions     FP64 -> FP32 and FP64 -> split BF16 operand copies.
#include "te_device.h"

#include <algorithm>

namespace te {
namespace {

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

// N uniform ints read at an index known only at run time. The selects keep
// them in scalar registers, where an indexed array would go to scratch memory.
template <int N> struct Sel {
  int c[N];
  __device__ int operator[](int q) const {
    int r = c[0];
#pragma unroll
    for (int m = 1; m < N; ++m) r = pick(q == m, c[m], r);
    return r;
  }
};

// One sextet as the kernel sees it: where its item's arrays are, which of the
// item's sextets it is, its box indices (A, B, C), the first slot holding each
// slot's box (slots repeat when A, B, C are not all different), and the
// occupied part of D. Everything here is uniform over the workgroup; slot s
// holds box (T[c_perm[s][0]], T[c_perm[s][1]], T[c_perm[s][2]]).
struct Sext {
  const void *W;
  const double *Kjk, *Kik, *Kij, *t1, *ev;
  double *part, *part5;
  long kld, local;
  int v, vp, nT, i, j, k;
  Sel<3> T;
  Sel<6> canon;
  double eijk;
};

// Read-only views in the constant address space: uniform loads through them
// become scalar loads, which the wave does not wait for at its vector-load
// counter (the next sextet's W loads stay in flight behind them).
template <typename T> using cptr = const __attribute__((address_space(4))) T *;

__device__ inline void sext_at(long g, const EItem *items, const int *blk_item,
                               int blks_per_item, long total, Sext &x) {
  int it;
  if (blk_item) {
    it = ((cptr<int>)blk_item)[g];
    x.local = g - ((cptr<int>)blk_item)[total + it];
  } else {
    it = (int)(g / blks_per_item);
    x.local = g - (long)it * blks_per_item;
  }
  cptr<EItem> e = (cptr<EItem>)items + it;
  x.W = e->W; x.Kjk = e->Kjk; x.Kik = e->Kik; x.Kij = e->Kij; x.kld = e->kld;
  x.t1 = e->t1; x.ev = e->ev; x.part = e->part; x.part5 = e->part5;
  x.v = e->v; x.vp = e->vp; x.nT = e->nT; x.i = e->i; x.j = e->j; x.k = e->k;
  const int packed = ((cptr<int>)e->sext)[x.local];
  x.T.c[0] = packed & 1023; x.T.c[1] = (packed >> 10) & 1023; x.T.c[2] = (packed >> 20) & 1023;
  int bx[6][3];
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    bx[s][0] = x.T[c_perm[s][0]]; bx[s][1] = x.T[c_perm[s][1]]; bx[s][2] = x.T[c_perm[s][2]];
    x.canon.c[s] = s;
#pragma unroll
    for (int q = 0; q < s; ++q)
      if (x.canon.c[s] == s && bx[q][0] == bx[s][0] && bx[q][1] == bx[s][1] &&
          bx[q][2] == bx[s][2])
        x.canon.c[s] = q;
  }
  cptr<double> eo = (cptr<double>)e->eo;
  x.eijk = (eo[x.i] + eo[x.j]) + eo[x.k];
}

// element u of a thread is element tid + 256 (u % 2) of slot u / 2
constexpr int EPER = 6 * BOX3 / WG;
constexpr int EKB = 3 * BOX * BOX, ENV = 4 * 3 * BOX;

// Issue the loads of one sextet: the inputs of V and D (per slot the 8 x 8
// blocks of (jb|kc), (ia|kc) and (ia|jb) it reads; per box index T[m] the
// eight t1 entries of rows i, j, k and the eight virtual orbital energies),
// then the three W shares of each distinct box. Box indices are below vp / 8, so
// every load is inside the padded arrays. Thread tid < EKB holds value tid of
// every slot's K blocks; the slot loop is unrolled and the box index chosen
// by selects, so that no private array is indexed per lane.
template <typename WT>
__device__ inline void sext_load(const Sext &x, int tid, WT (&w)[3][EPER], double (&kv)[6],
                                 double &tv) {
  {
    const int mat = tid >> 6, p = (tid >> 3) & 7, r = tid & 7;
    const double *Km = pick(mat == 0, x.Kjk, pick(mat == 1, x.Kik, x.Kij));
#pragma unroll
    for (int s = 0; s < 6; ++s) {
      kv[s] = 0.0;
      if (tid < EKB && x.canon.c[s] == s) {
        const int b0 = x.T[c_perm[s][0]], b1 = x.T[c_perm[s][1]], b2 = x.T[c_perm[s][2]];
        const int rb = pick(mat == 0, b1, b0);   // rows: b, a, a
        const int cb = pick(mat == 2, b1, b2);   // columns: c, c, b
        kv[s] = gld(Km + (long)(rb * BOX + p) * x.kld + cb * BOX + r);
      }
    }
  }
  tv = 0.0;
  if (tid < ENV) {
    const int wq = tid / (3 * BOX), m = (tid / BOX) % 3;
    const int xi = x.T[m] * BOX + (tid & 7);
    const int row = pick(wq == 0, x.i, pick(wq == 1, x.j, x.k));
    tv = wq == 3 ? gld(x.ev + xi) : gld(x.t1 + (long)row * x.vp + xi);
  }
  const long vp3 = (long)x.vp * x.vp * x.vp;
  const WT *W0 = reinterpret_cast<const WT *>(x.W);
  const WT *W1 = W0 + vp3;
  const WT *W2 = W1 + vp3;
#pragma unroll
  for (int u = 0; u < EPER; ++u) {
    const int s = u >> 1, r = tid + WG * (u & 1);
    w[0][u] = w[1][u] = w[2][u] = WT(0);
    if (x.canon.c[s] == s) {
      const int b0 = x.T[c_perm[s][0]], b1 = x.T[c_perm[s][1]], b2 = x.T[c_perm[s][2]];
      const long base = ((((long)b0 * x.nT + b1) * x.nT + b2) << 9) + r;
      w[0][u] = gld(W0 + base);
      w[1][u] = gld(W1 + base);
      w[2][u] = gld(W2 + base);
    }
  }
}

// Workgroup barrier ordering LDS accesses only: the wave waits for its own
// LDS accesses but not for its global loads (a __syncthreads would), so the
// next sextet's loads stay in flight across it.
__device__ inline void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Each workgroup evaluates es consecutive sextets of the launch's sextet list
// (global ids across items). The loads of sextet n+1 are issued right after
// sextet n is staged in LDS, so they are in flight while sextet n is
// evaluated from LDS. The arithmetic of each sextet, and its partial sums, do
// not depend on es.
template <typename WT>
__global__ __launch_bounds__(WG) void energy_kernel(const EItem *__restrict__ items,
                                                    const int *__restrict__ blk_item,
                                                    int blks_per_item, long total, int es) {
  __shared__ double box[6 * BX_S];
  __shared__ double kst[6 * EKB];
  __shared__ double vst[ENV];
  __shared__ double red[2 * (WG / 64)];
  const int tid = threadIdx.x;
  const long g0 = (long)blockIdx.x * es;
  const int cnt = (int)(total - g0 < es ? total - g0 : es);

  WT w[3][EPER];
  double kv[6], tv;
  Sext cur;
  sext_at(g0, items, blk_item, blks_per_item, total, cur);
  sext_load(cur, tid, w, kv, tv);

  for (int n = 0; n < cnt; ++n) {
    // stage sextet n: the three W shares summed into the padded boxes
#pragma unroll
    for (int u = 0; u < EPER; ++u) {
      const int s = u >> 1, r = tid + WG * (u & 1);
      if (cur.canon.c[s] == s)
        box[s * BX_S + bxi(r >> 6, (r >> 3) & 7, r & 7)] =
            ((double)w[0][u] + (double)w[1][u]) + (double)w[2][u];
    }
    if (tid < EKB) {
#pragma unroll
      for (int s = 0; s < 6; ++s) kst[s * EKB + tid] = kv[s];
    }
    if (tid < ENV) vst[tid] = tv;
    lds_barrier();

    Sext nxt = cur;
    if (n + 1 < cnt) {
      sext_at(g0 + n + 1, items, blk_item, blks_per_item, total, nxt);
      sext_load(nxt, tid, w, kv, tv);
    }

    const int v = cur.v;
    const Sel<3> &T = cur.T;
    const Sel<6> &canon = cur.canon;
    double acc4 = 0.0, acc5 = 0.0;   // W Z / D and V Z / D (E[4] and E[5] parts)
#pragma unroll 1
    for (int s = 0; s < 6; ++s) {
      if (canon[s] != s) continue;
      const int sb = canon[c_comp[s][3]] * BX_S;  // (b,c,a)
      const int sc = canon[c_comp[s][5]] * BX_S;  // (c,a,b)
      const int sd = canon[c_comp[s][1]] * BX_S;  // (a,c,b)
      const int se = canon[c_comp[s][2]] * BX_S;  // (b,a,c)
      const int sf = canon[c_comp[s][4]] * BX_S;  // (c,b,a)
      const double *ks = kst + s * EKB;
      const double *va = vst + c_perm[s][0] * BOX, *vb = vst + c_perm[s][1] * BOX,
                   *vc = vst + c_perm[s][2] * BOX;
      const int a0 = T[c_perm[s][0]] * 8, b0 = T[c_perm[s][1]] * 8, c0 = T[c_perm[s][2]] * 8;
      for (int r = tid; r < BOX3; r += WG) {
        const int x0 = r >> 6, x1 = (r >> 3) & 7, x2 = r & 7;
        const int a = a0 + x0, b = b0 + x1, c = c0 + x2;
        if (a < v && b < v && c < v) {
          const double w0 = box[s * BX_S + bxi(x0, x1, x2)];
          const double z = 4.0 * w0 + box[sb + bxi(x1, x2, x0)] + box[sc + bxi(x2, x0, x1)]
                           - 2.0 * box[sd + bxi(x0, x2, x1)] - 2.0 * box[se + bxi(x1, x0, x2)]
                           - 2.0 * box[sf + bxi(x2, x1, x0)];
          // singles term (Eq. 3): t_i^a (jb|kc) + t_j^b (ia|kc) + t_k^c (ia|jb)
          const double vt = va[x0] * ks[x1 * BOX + x2]
                          + vb[3 * BOX + x1] * ks[BOX * BOX + x0 * BOX + x2]
                          + vc[6 * BOX + x2] * ks[2 * BOX * BOX + x0 * BOX + x1];
          const double d = ((cur.eijk - va[9 * BOX + x0]) - vb[9 * BOX + x1]) - vc[9 * BOX + x2];
          const double q = z / d;
          acc4 += w0 * q;
          acc5 += vt * q;
        }
      }
    }
    // fixed-order reduction: butterfly within the wave, then waves in order
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      acc4 += __shfl_xor(acc4, off, 64);
      acc5 += __shfl_xor(acc5, off, 64);
    }
    if ((tid & 63) == 0) {
      red[tid >> 6] = acc4;
      red[WG / 64 + (tid >> 6)] = acc5;
    }
    // every wave is done with the boxes of sextet n past this barrier; thread
    // 0 reads red before it reaches the next one, and red is written again
    // only after it
    lds_barrier();
    if (tid == 0) {
      double s4 = red[0], s5 = red[WG / 64];
#pragma unroll
      for (int q = 1; q < WG / 64; ++q) {
        s4 += red[q];
        s5 += red[WG / 64 + q];
      }
      gst(cur.part + cur.local, s4);
      gst(cur.part5 + cur.local, s5);
    }
    cur = nxt;
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
  double x4 = 0.0, x5 = 0.0;
  for (int q = threadIdx.x; q < r.n; q += WG) {
    x4 += r.part[q];
    x5 += r.part5[q];
  }
  const double s4 = block_sum(x4, red);
  __syncthreads();                       // thread 0 has read red
  const double s5 = block_sum(x5, red);
  if (threadIdx.x == 0) {
    *r.out = r.w * (s4 + s5);
    if (r.out4) *r.out4 = r.w * s4;
    if (r.out5) *r.out5 = r.w * s5;
  }
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

// Independent products of one launch; grid layer z computes g[z].
struct GemmTNBatch {
  GemmTN g[3];
};

__global__ __launch_bounds__(WG) void gemm_tn_kernel(GemmTNBatch gb) {
  __shared__ __attribute__((aligned(16))) double As[GK][GT];
  __shared__ __attribute__((aligned(16))) double Bs[GK][GT];
  const GemmTN &g = gb.g[blockIdx.z];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.x * GT, n0 = blockIdx.y * GT;
  if (m0 >= g.M || n0 >= g.N) return;   // a layer smaller than the grid
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  d4 acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int r = 0; r < 4; ++r) acc[a][b][r] = 0.0;
  for (int k0 = 0; k0 < g.K; k0 += GK) {
    // a thread moves two consecutive elements of a k row, a wave two whole
    // rows: coalesced loads and 16-byte LDS stores that fill whole rows
    // (conflict-free); operands may sit at any 8-byte offset, so the global
    // loads stay element-wise
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      int e = tid + u * WG;
      int q = e >> 5, c = (e & 31) * 2;
      int kq = k0 + q;
      d2 a2, b2;
      a2[0] = (kq < g.K && m0 + c < g.M) ? g.A[(long)kq * g.lda + m0 + c] : 0.0;
      a2[1] = (kq < g.K && m0 + c + 1 < g.M) ? g.A[(long)kq * g.lda + m0 + c + 1] : 0.0;
      b2[0] = (kq < g.K && n0 + c < g.N) ? g.B[(long)kq * g.ldb + n0 + c] : 0.0;
      b2[1] = (kq < g.K && n0 + c + 1 < g.N) ? g.B[(long)kq * g.ldb + n0 + c + 1] : 0.0;
      *reinterpret_cast<d2 *>(&As[q][c]) = a2;
      *reinterpret_cast<d2 *>(&Bs[q][c]) = b2;
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
__device__ inline void split_store(double r, uint16_t *dst, size_t q, size_t n, int nparts) {
  for (int p = 0; p < nparts; ++p) {
    uint16_t h = bf16_rne((float)r);
    dst[p * n + q] = h;
    r -= bf16_val(h);
  }
}

// y = sigma x ~ h_0 + h_1 with h_0 = f16(y), h_1 = f16(y - h_0) (round to
// nearest even; sigma a power of two, so the scaling is exact); parts [2][n]
__device__ inline void split_store_f16(double x, uint16_t *dst, size_t q, size_t n, double sigma) {
  const double y = x * sigma;
  const _Float16 h0 = (_Float16)y;
  const _Float16 h1 = (_Float16)(y - (double)h0);
  dst[q] = __builtin_bit_cast(uint16_t, h0);
  dst[n + q] = __builtin_bit_cast(uint16_t, h1);
}

// parts stored [part][n]: BF16 (sigma == 0) or scaled FP16 (sigma != 0)
__global__ void to_bf16_parts_kernel(const double *__restrict__ src, uint16_t *__restrict__ dst,
                                     size_t n, int nparts, double sigma) {
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n;
       q += (size_t)gridDim.x * blockDim.x) {
    if (sigma != 0.0) split_store_f16(src[q], dst, q, n, sigma);
    else split_store(src[q], dst, q, n, nparts);
  }
}

// Panels of one occupied index p for a slice-cache slot, from its FP64
// column panel stg[l][a][b] = t2[l][p][a][b] (unpadded v, as copied from host
// memory), in the operand type of the W build and padded to vp like the
// resident arrays (same conversions, so the same bits):
//   col[part][l][a][b]      = t2[l][p][a][b]
//   row[l][a][b]            = t2[p][l][a][b] = stg[l][b][a]        (FP64, FP32)
//   row[part][y vp + z][l]  = t2[p][l][y][z] = stg[l][z][y], l < lo (BF16 parts)
__device__ inline void put(double *d, size_t q, size_t, double x, int) { d[q] = x; }
__device__ inline void put(float *d, size_t q, size_t, double x, int) { d[q] = (float)x; }
__device__ inline void put(uint16_t *d, size_t q, size_t n, double x, int np, double sigma) {
  if (sigma != 0.0) split_store_f16(x, d, q, n, sigma);
  else split_store(x, d, q, n, np);
}
__device__ inline void put(double *d, size_t q, size_t n, double x, int np, double) {
  put(d, q, n, x, np);
}
__device__ inline void put(float *d, size_t q, size_t n, double x, int np, double) {
  put(d, q, n, x, np);
}

// (16-bit parts: BF16 with sigma == 0, scaled FP16 otherwise)
template <typename OT>
__global__ void panel_kernel(const double *__restrict__ stg, OT *__restrict__ col,
                             OT *__restrict__ row, int o, int v, int vp, int lo, int nparts,
                             double sigma) {
  constexpr bool form = sizeof(OT) == 2;
  const long vp2 = (long)vp * vp;
  const size_t ncol = (size_t)o * vp2;
  const size_t nrow = form ? (size_t)vp2 * lo : ncol;
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < ncol + nrow;
       q += (size_t)gridDim.x * blockDim.x) {
    if (q < ncol) {
      const int b = (int)(q % vp);
      const size_t r = q / vp;
      const int a = (int)(r % vp), l = (int)(r / vp);
      const double x = (a < v && b < v) ? stg[((size_t)l * v + a) * v + b] : 0.0;
      put(col, q, ncol, x, nparts, sigma);
    } else if (form) {
      const size_t qq = q - ncol;
      const int l = (int)(qq % lo);
      const long pair = (long)(qq / lo);
      const int y = (int)(pair / vp), z = (int)(pair % vp);
      const double x = (l < o && y < v && z < v) ? stg[((size_t)l * v + z) * v + y] : 0.0;
      put(row, qq, nrow, x, nparts, sigma);
    } else {
      const size_t qq = q - ncol;
      const int b = (int)(qq % vp);
      const size_t r = qq / vp;
      const int a = (int)(r % vp), l = (int)(r / vp);
      const double x = (a < v && b < v) ? stg[((size_t)l * v + b) * v + a] : 0.0;
      put(row, qq, nrow, x, nparts, sigma);
    }
  }
}

__global__ void t2t_bf16_kernel(const double *__restrict__ t2, uint16_t *__restrict__ dst, int o,
                                int vp, int lo, int nparts, double sigma) {
  const long vp2 = (long)vp * vp;
  const size_t n = (size_t)o * vp2 * lo;
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n;
       q += (size_t)gridDim.x * blockDim.x) {
    const int l = (int)(q % lo);
    const size_t r = q / lo;
    const long pair = (long)(r % vp2);
    const int p = (int)(r / vp2);
    const double x = l < o ? t2[((long)p * o + l) * vp2 + pair] : 0.0;
    if (sigma != 0.0) split_store_f16(x, dst, q, n, sigma);
    else split_store(x, dst, q, n, nparts);
  }
}

__global__ void in_bf16_kernel(const double *__restrict__ in, uint16_t *__restrict__ dst, int o,
                               int vp, int lo, int nparts, double sigma) {
  const size_t n = (size_t)o * vp * o * lo;
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n;
       q += (size_t)gridDim.x * blockDim.x) {
    const int l = (int)(q % lo);
    const size_t r = q / lo;                  // (p, x, q') row
    const double x = l < o ? in[r * o + l] : 0.0;
    if (sigma != 0.0) split_store_f16(x, dst, q, n, sigma);
    else split_store(x, dst, q, n, nparts);
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

// max |x| over n doubles into *out (as the bit pattern of a non-negative
// double, which orders like an unsigned integer; *out starts at 0)
__global__ void absmax_kernel(const double *__restrict__ x, size_t n,
                              unsigned long long *out) {
  __shared__ double red[WG / 64];
  double m = 0.0;
  for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n;
       q += (size_t)gridDim.x * blockDim.x)
    m = fmax(m, fabs(x[q]));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < WG / 64; ++w) m = fmax(m, red[w]);
    atomicMax(out, (unsigned long long)__double_as_longlong(m));
  }
}

// max over columns c of sum_Q B[Q][c]^2, B stored [naux][ncol], into *out as
// absmax_kernel does
__global__ void colnorm_max_kernel(const double *__restrict__ B, int naux, long ncol,
                                   unsigned long long *out) {
  __shared__ double red[WG / 64];
  double m = 0.0;
  for (long c = blockIdx.x * (long)blockDim.x + threadIdx.x; c < ncol;
       c += (long)gridDim.x * blockDim.x) {
    double s2 = 0.0;
    for (int Q = 0; Q < naux; ++Q) {
      const double b = B[(long)Q * ncol + c];
      s2 += b * b;
    }
    m = fmax(m, s2);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < WG / 64; ++w) m = fmax(m, red[w]);
    atomicMax(out, (unsigned long long)__double_as_longlong(m));
  }
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

__global__ __launch_bounds__(WG) void probe_f16(float *out, int iters) {
  f4 acc[8];
  for (int c = 0; c < 8; ++c) acc[c] = f4{0, 0, 0, 0};
  h8 x, y;
  for (int e = 0; e < 8; ++e) {
    x[e] = (_Float16)(float)((threadIdx.x + e) & 7);
    y[e] = (_Float16)(float)(e - 3);
  }
  mfma_chains<h8, f4, 8>(x, y, acc, iters);
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
  else if (p == Prec::FP16X2) probe_f16<<<blocks, WG, 0, s>>>((float *)out, iters);
  else probe_bf16<<<blocks, WG, 0, s>>>((float *)out, iters);
  return hipGetLastError();
}

// ------------------------------------------------------------ launchers
hipError_t launch_energy(bool w_is_f64, const EItem *d_items, const int *d_blk_item, int nitems,
                         int blks_per_item, long total_blks, hipStream_t s) {
  (void)nitems;
  if (total_blks <= 0) return hipSuccess;
  if (total_blks > 0x7fffffffL) return hipErrorInvalidValue;
  // sextets per workgroup: 8, or fewer while that leaves under 4096
  // workgroups (about four per CU slot), so small launches still fill the chip
  const int es = (int)std::max(1L, std::min(8L, total_blks / 4096));
  dim3 grid((unsigned)((total_blks + es - 1) / es)), block(WG);
  if (w_is_f64)
    energy_kernel<double><<<grid, block, 0, s>>>(d_items, d_blk_item, blks_per_item, total_blks,
                                                 es);
  else
    energy_kernel<float><<<grid, block, 0, s>>>(d_items, d_blk_item, blks_per_item, total_blks,
                                                es);
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

hipError_t launch_gemm_tn_batch(const GemmTN *g, int n, hipStream_t s) {
  if (n < 1 || n > 3) return hipErrorInvalidValue;
  GemmTNBatch gb{};
  int mx = 0, nx = 0;
  for (int z = 0; z < n; ++z) {
    if (g[z].M <= 0 || g[z].N <= 0) return hipErrorInvalidValue;
    gb.g[z] = g[z];
    mx = std::max(mx, (g[z].M + GT - 1) / GT);
    nx = std::max(nx, (g[z].N + GT - 1) / GT);
  }
  dim3 grid(mx, nx, n);
  if (grid.y > 65535) return hipErrorInvalidValue;
  gemm_tn_kernel<<<grid, dim3(WG), 0, s>>>(gb);
  return hipGetLastError();
}

hipError_t launch_gemm_tn(const GemmTN &g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  return launch_gemm_tn_batch(&g, 1, s);
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
  to_bf16_parts_kernel<<<blocks_for(n), WG, 0, s>>>(src, dst, n, nparts, 0.0);
  return hipGetLastError();
}

hipError_t launch_panel(Prec p, const double *stg, void *col, void *row, int o, int v, int vp,
                        int lo, double sigma, hipStream_t s) {
  const size_t ncol = (size_t)o * vp * vp;
  const bool split = p == Prec::BF16X3 || p == Prec::BF16X2 || p == Prec::FP16X2;
  const size_t n = ncol + (split ? (size_t)vp * vp * lo : ncol);
  if (p == Prec::F64)
    panel_kernel<double><<<blocks_for(n), WG, 0, s>>>(stg, (double *)col, (double *)row, o, v,
                                                      vp, lo, 1, 0.0);
  else if (p == Prec::F32)
    panel_kernel<float><<<blocks_for(n), WG, 0, s>>>(stg, (float *)col, (float *)row, o, v, vp,
                                                     lo, 1, 0.0);
  else if (p == Prec::FP16X2)
    panel_kernel<uint16_t><<<blocks_for(n), WG, 0, s>>>(stg, (uint16_t *)col, (uint16_t *)row,
                                                        o, v, vp, lo, 2, sigma);
  else
    panel_kernel<uint16_t><<<blocks_for(n), WG, 0, s>>>(stg, (uint16_t *)col, (uint16_t *)row,
                                                        o, v, vp, lo,
                                                        p == Prec::BF16X2 ? 2 : 3, 0.0);
  return hipGetLastError();
}

hipError_t launch_to_f16_parts(const double *src, uint16_t *dst, size_t n, double sigma,
                               hipStream_t s) {
  to_bf16_parts_kernel<<<blocks_for(n), WG, 0, s>>>(src, dst, n, 2, sigma);
  return hipGetLastError();
}

hipError_t launch_t2t_f16_parts(const double *t2, uint16_t *dst, int o, int vp, int lo,
                                double sigma, hipStream_t s) {
  size_t n = (size_t)o * vp * vp * lo;
  t2t_bf16_kernel<<<blocks_for(n), WG, 0, s>>>(t2, dst, o, vp, lo, 2, sigma);
  return hipGetLastError();
}

hipError_t launch_in_f16_parts(const double *in, uint16_t *dst, int o, int vp, int lo,
                               double sigma, hipStream_t s) {
  size_t n = (size_t)o * vp * o * lo;
  in_bf16_kernel<<<blocks_for(n), WG, 0, s>>>(in, dst, o, vp, lo, 2, sigma);
  return hipGetLastError();
}

hipError_t launch_absmax(const double *x, size_t n, unsigned long long *out, hipStream_t s) {
  absmax_kernel<<<blocks_for(n), WG, 0, s>>>(x, n, out);
  return hipGetLastError();
}

hipError_t launch_colnorm_max(const double *B, int naux, long ncol, unsigned long long *out,
                              hipStream_t s) {
  colnorm_max_kernel<<<blocks_for((size_t)ncol), WG, 0, s>>>(B, naux, ncol, out);
  return hipGetLastError();
}

hipError_t launch_t2t_bf16_parts(const double *t2, uint16_t *dst, int o, int vp, int lo,
                                 int nparts, hipStream_t s) {
  size_t n = (size_t)o * vp * vp * lo;
  t2t_bf16_kernel<<<blocks_for(n), WG, 0, s>>>(t2, dst, o, vp, lo, nparts, 0.0);
  return hipGetLastError();
}

hipError_t launch_in_bf16_parts(const double *in, uint16_t *dst, int o, int vp, int lo,
                                int nparts, hipStream_t s) {
  size_t n = (size_t)o * vp * o * lo;
  in_bf16_kernel<<<blocks_for(n), WG, 0, s>>>(in, dst, o, vp, lo, nparts, 0.0);
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
