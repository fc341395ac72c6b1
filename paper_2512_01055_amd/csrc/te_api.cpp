// C-ABI host side of the (T) library: validation, staging of the padded
// device layouts, precision copies, triple scheduling and launch ordering.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <map>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "te.h"
#include "te_internal.h"
#include "te_job.h"

namespace te {

thread_local std::string g_last_error;

Fail::Fail(te_status s_, std::string m) : s(s_), msg(std::move(m)) {}

void hip_check(hipError_t e, const char *what, int line) {
  if (e != hipSuccess)
    throw Fail(TE_EDEVICE, std::string(what) + " (line " + std::to_string(line) +
                               "): " + hipGetErrorString(e));
}

te_status set_error(te_status s, const std::string &m) {
  g_last_error = m;
  return s;
}

// ------------------------------------------------------------ Arena
void Arena::init(size_t bytes) {
  bytes = (bytes + 255) & ~(size_t)255;
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess)
    throw Fail(TE_ENOMEM, "arena hipMalloc(" + std::to_string(bytes) + "): " + hipGetErrorString(e));
  base = (char *)p;
  cap = bytes;
  used = 0;
  free_.clear();
  free_[0] = bytes;
}
void Arena::destroy() {
  if (base) (void)hipFree(base);
  base = nullptr;
  cap = used = 0;
  free_.clear();
}
void *Arena::take(size_t n) {
  std::lock_guard<std::mutex> lk(mu);
  n = (n + 255) & ~(size_t)255;
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second >= n) {
      size_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > n) free_[off + n] = len - n;
      used += n;
      return base + off;
    }
  }
  return nullptr;
}
void Arena::give(void *p, size_t n) {
  std::lock_guard<std::mutex> lk(mu);
  n = (n + 255) & ~(size_t)255;
  size_t off = (size_t)((char *)p - base);
  used -= n;
  auto it = free_.emplace(off, n).first;
  auto nx = std::next(it);
  if (nx != free_.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    free_.erase(nx);
  }
  if (it != free_.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      free_.erase(it);
    }
  }
}
size_t Arena::largest_free() {
  std::lock_guard<std::mutex> lk(mu);
  size_t m = 0;
  for (auto &kv : free_) m = std::max(m, kv.second);
  return m;
}

// ------------------------------------------------------------ DBuf
DBuf::~DBuf() { release(); }
void DBuf::release() {
  if (p) {
    if (arena) arena->give(p, bytes);
    else (void)hipFree(p);
  }
  if (acct) *acct -= bytes;
  p = nullptr;
  bytes = 0;
  acct = nullptr;
  arena = nullptr;
}
void DBuf::alloc(size_t n, size_t *account, size_t budget, Arena *ar) {
  release();
  if (n == 0) n = 16;
  if (account && *account + n > budget)
    throw Fail(TE_ENOMEM, "device allocation of " + std::to_string(n) +
                              " bytes exceeds the HBM budget (" + std::to_string(*account) +
                              " of " + std::to_string(budget) + " in use)");
  if (ar) {
    p = ar->take(n);
    if (!p)
      throw Fail(TE_ENOMEM, "arena has no free range of " + std::to_string(n) + " bytes");
  } else {
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
      p = nullptr;
      throw Fail(TE_ENOMEM, "hipMalloc(" + std::to_string(n) + "): " + hipGetErrorString(e));
    }
  }
  bytes = n;
  acct = account;
  arena = ar;
  if (acct) *acct += n;
}

void jalloc(Job &J, DBuf &b, size_t n) { b.alloc(n, &J.used, J.budget, J.arena); }

// ------------------------------------------------------------ triples
std::vector<int> triple_list_host(int o) {
  std::vector<int> t;
  for (int i = 0; i < o; ++i)
    for (int j = i; j < o; ++j)
      for (int k = j; k < o; ++k)
        if (!(i == j && j == k)) { t.push_back(i); t.push_back(j); t.push_back(k); }
  return t;
}

std::vector<int> sextet_list(int nT) {
  std::vector<int> s;
  s.reserve((size_t)nT * (nT + 1) * (nT + 2) / 6);
  for (int A = 0; A < nT; ++A)
    for (int B = 0; B <= A; ++B)
      for (int C = 0; C <= B; ++C) s.push_back(A | (B << 10) | (C << 20));
  return s;
}

static size_t elem_size(Prec p) {
  return p == Prec::F64 ? 8 : (p == Prec::F32 ? 4 : 2);
}
static int nparts(Prec p) {
  return p == Prec::BF16X3 ? 3 : (p == Prec::BF16X2 || p == Prec::FP16X2 ? 2 : 1);
}
static size_t out_size(Prec p) { return p == Prec::F64 ? 8 : 4; }

// ------------------------------------------------------------ staging
static void copy_in(Job &J, const double *src, size_t n, DBuf &dst, bool device_src) {
  jalloc(J, dst, n * sizeof(double));
  HIPCHK(hipMemcpyAsync(dst.p, src, n * sizeof(double),
                        device_src ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, J.s_main));
}

// Make a device-resident unpadded copy (or borrow a device pointer).
static const double *device_view(Job &J, const double *src, size_t n, DBuf &tmp) {
  if (J.mem == TE_MEM_DEVICE) return src;
  copy_in(J, src, n, tmp, false);
  return tmp.as<double>();
}

static void stage_padded(Job &J, const double *src, int d0, int d1, int d2, int d3, int p1,
                         int p2, int p3, double scale, DBuf &dst) {
  size_t n = (size_t)d0 * p1 * p2 * p3;
  jalloc(J, dst, n * sizeof(double));
  HIPCHK(hipMemsetAsync(dst.p, 0, n * sizeof(double), J.s_main));
  DBuf tmp;
  const double *s = device_view(J, src, (size_t)d0 * d1 * d2 * d3, tmp);
  HIPCHK(launch_pad4(s, dst.as<double>(), d0, d1, d2, d3, p1, p2, p3, scale, J.s_main));
  if (tmp.p) HIPCHK(hipStreamSynchronize(J.s_main));
}

// Largest |x| over n device doubles, and the largest column norm^2 of a
// factor [naux][ncol]; both synchronous (set-up only).
static double read_max(Job &J, DBuf &m) {
  unsigned long long bits = 0;
  HIPCHK(hipMemcpyAsync(&bits, m.p, 8, hipMemcpyDeviceToHost, J.s_main));
  HIPCHK(hipStreamSynchronize(J.s_main));
  double r;
  std::memcpy(&r, &bits, 8);
  return r;
}
static double dev_absmax(Job &J, const double *x, size_t n) {
  if (!x || !n) return 0.0;
  DBuf m;
  m.alloc(8, nullptr, 0);
  HIPCHK(hipMemsetAsync(m.p, 0, 8, J.s_main));
  HIPCHK(launch_absmax(x, n, m.as<unsigned long long>(), J.s_main));
  return read_max(J, m);
}
static double dev_colnorm_max(Job &J, const double *B, long ncol) {
  if (!B || ncol <= 0) return 0.0;
  DBuf m;
  m.alloc(8, nullptr, 0);
  HIPCHK(hipMemsetAsync(m.p, 0, 8, J.s_main));
  HIPCHK(launch_colnorm_max(B, J.naux, ncol, m.as<unsigned long long>(), J.s_main));
  return read_max(J, m);
}
// Largest |x| over n host doubles, on a few threads.
static double host_absmax(const double *x, size_t n) {
  const size_t nth = std::max(1u, std::min(8u, std::thread::hardware_concurrency()));
  std::vector<double> part(nth, 0.0);
  auto run = [&](size_t t) {
    double m = 0.0;
    for (size_t q = t * n / nth, e = (t + 1) * n / nth; q < e; ++q) m = std::max(m, std::abs(x[q]));
    part[t] = m;
  };
  std::vector<std::thread> th;
  for (size_t t = 1; t < nth; ++t) th.emplace_back(run, t);
  run(0);
  for (auto &x_ : th) x_.join();
  return *std::max_element(part.begin(), part.end());
}

// 2^k with k the largest integer such that 2^k m <= 2^14 (1 for m = 0)
static double pow2_scale(double m) {
  if (!(m > 0.0) || !std::isfinite(m)) return 1.0;
  return std::ldexp(1.0, (int)std::floor(std::log2(16384.0 / m)));
}

static void gemm_stage(Job &J, const double *A, long lda, const double *B, long ldb, int M,
                       int N, int K, int rd, long rs1, long rs2, int cd, long cs1, long cs2,
                       double alpha, double *C) {
  GemmTN g{A, B, C, M, N, K, lda, ldb, rd, rs1, rs2, cd, cs1, cs2, alpha};
  HIPCHK(launch_gemm_tn(g, J.s_main));
}

void stage_df_slices(Job &J, const int *occ, int n, double *dst, size_t slice_stride) {
  // X_p[x][y][f] = (px|yf) = sum_Q B^Q_px B^Q_yf   (Eq. 6)
  const int o = J.o, v = J.v, vp = J.vp, naux = J.naux;
  const long vp2 = (long)vp * vp;
  for (int q = 0; q < n; ++q) {
    double *C = dst + (size_t)q * slice_stride;
    if (v != vp) HIPCHK(hipMemsetAsync(C, 0, (size_t)vp2 * vp * sizeof(double), J.s_main));
    gemm_stage(J, J.Bov + (long)occ[q] * v, (long)o * v, J.Bvv, (long)v * v, v, v * v, naux,
               v, vp2, vp2, v, vp, 1, 1.0, C);
  }
}

static void stage(Job &J, const te_problem &P) {
  const int o = J.o, v = J.v, vp = J.vp;
  const bool dev = P.mem == TE_MEM_DEVICE;
  hipStream_t s = J.s_main;

  // orbital energies and singles, padded in v
  copy_in(J, P.eps_occ, o, J.eo, dev);
  {
    DBuf tmp;
    const double *ev = device_view(J, P.eps_vir, v, tmp);
    jalloc(J, J.ev, (size_t)vp * 8);
    HIPCHK(hipMemsetAsync(J.ev.p, 0, (size_t)vp * 8, s));
    HIPCHK(hipMemcpyAsync(J.ev.p, ev, (size_t)v * 8, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  stage_padded(J, P.t1, 1, 1, o, v, 1, o, vp, 1.0, J.t1);

  // doubles: borrowed when already in device memory with an aligned v; left
  // in host memory in the host-t2 mode (panels go to the slice cache)
  if (J.t2h) {
    J.t2 = nullptr;
  } else if (dev && vp == v) {
    J.t2 = P.t2;
  } else {
    stage_padded(J, P.t2, o, o, v, v, o, vp, vp, 1.0, J.t2_own);
    J.t2 = J.t2_own.as<double>();
  }

  const size_t nX = (size_t)o * vp * vp * vp;
  if (J.naux > 0) {
    const int naux = J.naux;
    if (J.x_resident) {
      // read only here: device arrays are borrowed for the call
      J.Bov = device_view(J, P.B_ov, (size_t)naux * o * v, J.Bov_own);
      J.Bvv = device_view(J, P.B_vv, (size_t)naux * v * v, J.Bvv_own);
    } else {
      // on the fly, every later call assembles slices and (ov|ov) blocks
      // from B_ov and B_vv: the job keeps its own copies, so the caller may
      // free device arrays once te_init returns
      copy_in(J, P.B_ov, (size_t)naux * o * v, J.Bov_own, dev);
      copy_in(J, P.B_vv, (size_t)naux * v * v, J.Bvv_own, dev);
      J.Bov = J.Bov_own.as<double>();
      J.Bvv = J.Bvv_own.as<double>();
    }
    J.Boo = device_view(J, P.B_oo, (size_t)naux * o * o, J.Boo_own);
    // |(px|yf)| <= |B_px| |B_yf| (Cauchy-Schwarz over the factor index)
    J.x_bound = std::sqrt(dev_colnorm_max(J, J.Bov, (long)o * v) *
                          dev_colnorm_max(J, J.Bvv, (long)v * v));
    // K[p][x][q][y] = (px|qy), for V (Eq. 3); when (vv|vo) is assembled on
    // the fly the three blocks a triple reads are assembled with it instead
    if (J.x_resident) {
      jalloc(J, J.K, (size_t)o * vp * o * vp * 8);
      HIPCHK(hipMemsetAsync(J.K.p, 0, J.K.bytes, s));
      gemm_stage(J, J.Bov, (long)o * v, J.Bov, (long)o * v, o * v, o * v, naux, v,
                 (long)vp * o * vp, (long)o * vp, v, vp, 1, 1.0, J.K.as<double>());
    }
    // In[p][x][q][l] = -(px|ql), the occupied term of Eq. 2 with its sign
    jalloc(J, J.In, (size_t)o * vp * o * o * 8);
    HIPCHK(hipMemsetAsync(J.In.p, 0, J.In.bytes, s));
    gemm_stage(J, J.Bov, (long)o * v, J.Boo, (long)o * o, o * v, o * o, naux, v,
               (long)vp * o * o, (long)o * o, o * o, 0, 1, -1.0, J.In.as<double>());
    HIPCHK(hipStreamSynchronize(s));
    J.Boo_own.release();            // B_oo is not read after staging
    J.Boo = nullptr;
    if (J.x_resident) {
      jalloc(J, J.X, nX * 8);
      std::vector<int> all(o);
      for (int p = 0; p < o; ++p) all[p] = p;
      stage_df_slices(J, all.data(), o, J.X.as<double>(), (size_t)vp * vp * vp);
      HIPCHK(hipStreamSynchronize(s));
      // factors are no longer needed once every slice is resident
      J.Bov_own.release(); J.Bvv_own.release();
      J.Bov = J.Bvv = nullptr;
    }
  } else {
    stage_padded(J, P.ovov, o, v, o, v, vp, o, vp, 1.0, J.K);
    stage_padded(J, P.ovoo, o, v, o, o, vp, o, o, -1.0, J.In);
    stage_padded(J, P.ovvv, o, v, v, v, vp, vp, vp, 1.0, J.X);
  }
  HIPCHK(hipStreamSynchronize(s));
}

static void validate_device(Job &J, const te_problem &P) {
  // non-finite values anywhere in the staged data, and t2 pair symmetry
  DBuf flag;
  flag.alloc(64, nullptr, 0);
  HIPCHK(hipMemsetAsync(flag.p, 0, 64, J.s_main));
  auto chk = [&](const void *p, size_t n) {
    if (p && n) HIPCHK(launch_check((const double *)p, n, flag.as<int>(), J.s_main));
  };
  chk(J.eo.p, J.eo.bytes / 8);
  chk(J.ev.p, J.ev.bytes / 8);
  chk(J.t1.p, J.t1.bytes / 8);
  if (J.t2) chk(J.t2, (size_t)J.o * J.o * J.vp * J.vp);
  chk(J.K.p, J.K.bytes / 8);
  chk(J.In.p, J.In.bytes / 8);
  chk(J.X.p, J.X.bytes / 8);
  if (J.t2)
    HIPCHK(launch_t2_asym(J.t2, J.o, J.vp, (double *)(flag.as<char>() + 16), nullptr, J.s_main));
  int bad = 0;
  double mm[2] = {0, 0};
  HIPCHK(hipMemcpyAsync(&bad, flag.p, 4, hipMemcpyDeviceToHost, J.s_main));
  HIPCHK(hipMemcpyAsync(mm, flag.as<char>() + 16, 16, hipMemcpyDeviceToHost, J.s_main));
  HIPCHK(hipStreamSynchronize(J.s_main));
  (void)P;
  if (bad) throw Fail(TE_EINVAL, "input holds a non-finite value");
  if (mm[0] > 1e-12 * std::max(mm[1], 1e-300))
    throw Fail(TE_EINVAL, "t2 is not pair-symmetric: max |t_ij^ab - t_ji^ba| = " +
                              std::to_string(mm[0]));
}

// ------------------------------------------------------------ precisions
static void drop_operands(Operands &op) {
  op.X_own.release(); op.T2_own.release(); op.In_own.release(); op.T2T_own.release();
  op.ready = false;
  op.X = op.T2 = op.In = op.T2T = nullptr;
  op.xps = op.tps = op.ips = op.t2tps = 0;
  op.lo = 0;
  op.scale = 1.0f;
  op.sigma_x = op.sigma_t = 1.0;
}

const Operands &ensure_prec(Job &J, Prec p) {
  const int slot = (int)p;
  Operands &op = J.op[slot];
  if (op.ready) return op;
  // at most one reduced-precision copy at a time: it is rebuilt from the
  // FP64 arrays in milliseconds, and the HBM goes to the slice cache
  if (p != Prec::F64) {
    HIPCHK(hipStreamSynchronize(J.s_main));
    if (J.s_aux) HIPCHK(hipStreamSynchronize(J.s_aux));
    for (int q : {(int)Prec::F32, (int)Prec::BF16X3, (int)Prec::BF16X2, (int)Prec::FP16X2})
      if (q != slot) drop_operands(J.op[q]);
  }
  const int o = J.o, vp = J.vp;
  const size_t nT2 = (size_t)o * o * vp * vp;
  const size_t nIn = (size_t)o * vp * o * o;
  const size_t nX = J.X.p ? (size_t)o * vp * vp * vp : 0;
  if (p != Prec::F64 && !J.X.p && J.x_resident)
    throw Fail(TE_EINVAL, "the FP64 (vv|vo) copy was released; precision cannot change");
  op.lo = o;
  if (p == Prec::F64) {
    if (!J.X.p && J.x_resident)
      throw Fail(TE_EINVAL, "the FP64 (vv|vo) copy was released; precision cannot change");
    op.X = J.X.p; op.T2 = J.t2; op.In = J.In.p;
    op.xps = nX; op.tps = nT2; op.ips = nIn;
  } else if (p == Prec::F32) {
    if (J.t2) {    // (host t2: panels are converted as they enter the slice cache)
      jalloc(J, op.T2_own, nT2 * 4);
      HIPCHK(launch_to_f32(J.t2, op.T2_own.as<float>(), nT2, J.s_main));
    }
    jalloc(J, op.In_own, nIn * 4);
    HIPCHK(launch_to_f32(J.In.as<double>(), op.In_own.as<float>(), nIn, J.s_main));
    if (nX) {
      jalloc(J, op.X_own, nX * 4);
      HIPCHK(launch_to_f32(J.X.as<double>(), op.X_own.as<float>(), nX, J.s_main));
    }
    op.X = op.X_own.p; op.T2 = op.T2_own.p; op.In = op.In_own.p;
    op.xps = nX; op.tps = nT2; op.ips = nIn;
  } else if (p == Prec::FP16X2) {
    // two FP16 parts of sigma x; sigma_x scales X and In (their products with
    // t2 share one accumulator), sigma_t scales t2, each bringing the largest
    // magnitude to at most 2^14 (FP16 holds up to 65504)
    const int lo = (o + 7) / 8 * 8;
    const size_t nInP = (size_t)o * vp * o * lo, nT2T = (size_t)o * vp * vp * lo;
    double mx = dev_absmax(J, J.In.as<double>(), nIn);
    if (J.naux > 0) {
      // the factor bound, the same whether the slices are resident or
      // assembled on the fly
      mx = std::max(mx, J.x_bound);
    } else {
      mx = std::max(mx, dev_absmax(J, J.X.as<double>(), nX));
    }
    op.sigma_x = pow2_scale(mx);
    // (host t2: the same maximum, taken on the host; its panels are scaled
    // as they enter the slice cache)
    op.sigma_t = pow2_scale(J.t2 ? dev_absmax(J, J.t2, nT2) : host_absmax(J.t2h, (size_t)o * o * J.v * J.v));
    op.scale = (float)(1.0 / (op.sigma_x * op.sigma_t));
    jalloc(J, op.In_own, nInP * 2 * 2);
    HIPCHK(launch_in_f16_parts(J.In.as<double>(), op.In_own.as<uint16_t>(), o, vp, lo,
                               op.sigma_x, J.s_main));
    if (J.t2) {
      jalloc(J, op.T2_own, nT2 * 2 * 2);
      jalloc(J, op.T2T_own, nT2T * 2 * 2);
      HIPCHK(launch_to_f16_parts(J.t2, op.T2_own.as<uint16_t>(), nT2, op.sigma_t, J.s_main));
      HIPCHK(launch_t2t_f16_parts(J.t2, op.T2T_own.as<uint16_t>(), o, vp, lo, op.sigma_t,
                                  J.s_main));
    }
    if (nX) {
      jalloc(J, op.X_own, nX * 2 * 2);
      HIPCHK(launch_to_f16_parts(J.X.as<double>(), op.X_own.as<uint16_t>(), nX, op.sigma_x,
                                 J.s_main));
    }
    op.X = op.X_own.p; op.T2 = op.T2_own.p; op.In = op.In_own.p; op.T2T = op.T2T_own.p;
    op.xps = nX; op.tps = nT2; op.ips = nInP; op.t2tps = nT2T; op.lo = lo;
  } else {
    // BF16 parts (three, or the first two of the same split); the
    // occupied-index operands get l last and padded to 8 so the W build loads
    // them as 16-byte chunks
    const int np = nparts(p);
    const int lo = (o + 7) / 8 * 8;
    const size_t nInP = (size_t)o * vp * o * lo, nT2T = (size_t)o * vp * vp * lo;
    jalloc(J, op.In_own, nInP * 2 * np);
    HIPCHK(launch_in_bf16_parts(J.In.as<double>(), op.In_own.as<uint16_t>(), o, vp, lo, np,
                                J.s_main));
    if (J.t2) {
      jalloc(J, op.T2_own, nT2 * 2 * np);
      jalloc(J, op.T2T_own, nT2T * 2 * np);
      HIPCHK(launch_to_bf16_parts(J.t2, op.T2_own.as<uint16_t>(), nT2, np, J.s_main));
      HIPCHK(launch_t2t_bf16_parts(J.t2, op.T2T_own.as<uint16_t>(), o, vp, lo, np, J.s_main));
    }
    if (nX) {
      jalloc(J, op.X_own, nX * 2 * np);
      HIPCHK(launch_to_bf16_parts(J.X.as<double>(), op.X_own.as<uint16_t>(), nX, np, J.s_main));
    }
    op.X = op.X_own.p; op.T2 = op.T2_own.p; op.In = op.In_own.p; op.T2T = op.T2T_own.p;
    op.xps = nX; op.tps = nT2; op.ips = nInP; op.t2tps = nT2T; op.lo = lo;
  }
  HIPCHK(hipStreamSynchronize(J.s_main));
  op.ready = true;
  return op;
}

// ------------------------------------------------------------ execution
// Pairs of events bracketing each launch of one kernel.
struct TimingEvents {
  std::vector<hipEvent_t> start, stop;
  explicit TimingEvents(long n) : start(n, nullptr), stop(n, nullptr) {
    for (long q = 0; q < n; ++q) {
      HIPCHK(hipEventCreate(&start[q]));
      HIPCHK(hipEventCreate(&stop[q]));
    }
  }
  ~TimingEvents() {
    for (auto e : start) if (e) (void)hipEventDestroy(e);
    for (auto e : stop) if (e) (void)hipEventDestroy(e);
  }
  double total() const {  // seconds; call after the stream has been synchronised
    double s = 0.0;
    for (size_t q = 0; q < start.size(); ++q) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, start[q], stop[q]) == hipSuccess) s += ms * 1e-3;
    }
    return s;
  }
};

double flops_per_triple(int o, int v) { return 12.0 * (double)v * v * v * ((double)v + o); }

// Triples per launch: at least 64k workgroup tiles (about 85 waves of
// workgroups over the chip), so that the last, partly filled wave of a
// launch costs little. The W scratch of one batch stays within 8 GB, a
// sixteenth of the budget, and a 64th of the W of all the call's triples
// (but may take 256 MB): allocating (and freeing) scratch costs about 12 ms
// per GB, which a small job's whole evaluation would not cover (o=16, v=128
// took three times as long with 16 GB of scratch).
static int batch_size(const Job &J, Prec p, long ntr) {
  const WConfig wc = wbuild_config(p, J.vp);
  const long mt = ((long)J.vp * J.vp + wc.bm() - 1) / wc.bm();
  const long nt = (J.vp + wc.bn() - 1) / wc.bn();
  const long tiles = 3 * mt * nt;
  long b = std::max(1L, (65536 + tiles - 1) / tiles);
  const size_t per = 3 * (size_t)J.vp * J.vp * J.vp * out_size(p);
  const size_t cap = std::max<size_t>(
      per, std::min({(size_t)8 << 30, J.budget / 16,
                     std::max<size_t>((size_t)ntr * per / 64, (size_t)256 << 20)}));
  b = std::min<long>(b, std::max<long>(1, (long)(cap / per)));
  b = std::min<long>(b, ntr);
  return (int)std::max(1L, b);
}

// Execution plan for a list of triples: the order they run in, the batches,
// and (on-the-fly mode) which (vv|vo) slice sits in which cache slot.
struct Plan {
  std::vector<long> order;                               // position -> caller index
  std::vector<long> bfirst;                              // batch -> first position
  std::vector<int> bcount;
  std::vector<std::vector<std::pair<int, int>>> loads;   // batch -> (occupied p, slot)
  std::vector<std::array<int, 3>> slot;                  // position -> slots of X_i, X_j, X_k
  long nloads = 0;
};

static Plan plan_resident(long ntr, int B) {
  Plan P;
  P.order.resize(ntr);
  for (long t = 0; t < ntr; ++t) P.order[t] = t;
  for (long f = 0; f < ntr; f += B) {
    P.bfirst.push_back(f);
    P.bcount.push_back((int)std::min<long>(B, ntr - f));
  }
  P.loads.resize(P.bfirst.size());
  return P;
}

// Occupied indices are grouped in blocks of S/3; triples run block-triple by
// block-triple so that a cache of S slices is refilled about once per block
// change. Within a batch every needed slice is resident; misses evict the
// least recently used slice not needed by the batch. `held` gives the slot
// contents on entry (-1: empty) and receives them on return.
static Plan plan_on_the_fly(const int *ijk, long ntr, int B, std::vector<int> &held) {
  const int S = (int)held.size();
  Plan P;
  const int bs = std::max(1, S / 3);
  P.order.resize(ntr);
  for (long t = 0; t < ntr; ++t) P.order[t] = t;
  std::stable_sort(P.order.begin(), P.order.end(), [&](long a, long b) {
    const int *x = ijk + 3 * a, *y = ijk + 3 * b;
    for (int d = 0; d < 3; ++d)
      if (x[d] / bs != y[d] / bs) return x[d] / bs < y[d] / bs;
    for (int d = 0; d < 3; ++d)
      if (x[d] != y[d]) return x[d] < y[d];
    return false;
  });
  std::vector<long> last(S, -1);       // slot -> last batch that used it
  std::map<int, int> where;            // occupied index -> slot
  for (int q = 0; q < S; ++q)
    if (held[q] >= 0) where[held[q]] = q;
  P.slot.resize(ntr);
  long pos = 0, bno = 0;
  while (pos < ntr) {
    std::vector<int> need;
    auto has = [&](int p) { return std::find(need.begin(), need.end(), p) != need.end(); };
    long end = pos;
    while (end < ntr && end - pos < B) {
      const int *x = ijk + 3 * P.order[end];
      std::vector<int> add;
      for (int d = 0; d < 3; ++d)
        if (!has(x[d]) && std::find(add.begin(), add.end(), x[d]) == add.end()) add.push_back(x[d]);
      if ((int)(need.size() + add.size()) > S) break;
      need.insert(need.end(), add.begin(), add.end());
      ++end;
    }
    std::vector<std::pair<int, int>> loads;
    for (int p : need) {
      auto it = where.find(p);
      if (it != where.end()) { last[it->second] = bno; continue; }
      int victim = -1;
      for (int q = 0; q < S; ++q) {
        if (held[q] >= 0 && has(held[q])) continue;
        if (victim < 0 || last[q] < last[victim]) victim = q;
      }
      if (held[victim] >= 0) where.erase(held[victim]);
      held[victim] = p;
      where[p] = victim;
      last[victim] = bno;
      loads.push_back({p, victim});
    }
    for (long q = pos; q < end; ++q) {
      const int *x = ijk + 3 * P.order[q];
      P.slot[q] = {where[x[0]], where[x[1]], where[x[2]]};
    }
    P.bfirst.push_back(pos);
    P.bcount.push_back((int)(end - pos));
    P.loads.push_back(loads);
    P.nloads += (long)loads.size();
    pos = end;
    ++bno;
  }
  return P;
}

// Assemble X_p[x][y][f] = (px|yf) = sum_Q B^Q_px B^Q_yf (Eq. 6) into a cache
// slot, in the precision the W build reads.
static void assemble_slice(Job &J, Prec p, int occ, void *slot, double *tmp64, hipStream_t s) {
  const int o = J.o, v = J.v, vp = J.vp, naux = J.naux;
  const long vp2 = (long)vp * vp;
  const size_t n = (size_t)vp2 * vp;
  double *dst = p == Prec::F64 ? (double *)slot : tmp64;
  // the product writes every element unless v is padded; padding must read 0
  if (v != vp) HIPCHK(hipMemsetAsync(dst, 0, n * sizeof(double), s));
  GemmTN g{J.Bov + (long)occ * v, J.Bvv, dst, v, v * v, naux, (long)o * v, (long)v * v,
           v, vp2, vp2, v, vp, 1, 1.0};
  HIPCHK(launch_gemm_tn(g, s));
  if (p == Prec::F32) HIPCHK(launch_to_f32(tmp64, (float *)slot, n, s));
  if (p == Prec::BF16X3 || p == Prec::BF16X2)
    HIPCHK(launch_to_bf16_parts(tmp64, (uint16_t *)slot, n, nparts(p), s));
  if (p == Prec::FP16X2)
    HIPCHK(launch_to_f16_parts(tmp64, (uint16_t *)slot, n, J.op[(int)Prec::FP16X2].sigma_x, s));
}

// Host t2: the column panel t2[:, occ] is gathered into the pinned bounce
// buffer (once the previous copy out of it has completed), copied to the
// device on stream s, and expanded by the panel kernel into a cache slot's
// column panel and row panel / row form, in the precision the W build reads.
static void fill_panels(Job &J, Prec p, int occ, char *col, char *row, hipStream_t s) {
  const size_t o = J.o, v2 = (size_t)J.v * J.v;
  const int x = J.xc.nfill++ & 1;
  double *pinned = J.xc.pinned[x];
  HIPCHK(hipEventSynchronize(J.xc.pinned_free[x]));
  // the o blocks t2[l][occ] are independent: gather them on a few threads
  const size_t nth = std::min<size_t>(o, std::max(1u, std::min(8u, std::thread::hardware_concurrency())));
  auto gather = [&](size_t t) {
    for (size_t l = t; l < o; l += nth)
      std::memcpy(pinned + l * v2, J.t2h + (l * o + (size_t)occ) * v2, v2 * 8);
  };
  std::vector<std::thread> th;
  for (size_t t = 1; t < nth; ++t) th.emplace_back(gather, t);
  gather(0);
  for (auto &x : th) x.join();
  HIPCHK(hipMemcpyAsync(J.xc.tstg.p, pinned, o * v2 * 8, hipMemcpyHostToDevice, s));
  HIPCHK(hipEventRecord(J.xc.pinned_free[x], s));
  const int lo = p == Prec::F64 || p == Prec::F32 ? J.o : (J.o + 7) / 8 * 8;
  HIPCHK(launch_panel(p, J.xc.tstg.as<double>(), col, row, J.o, J.v, J.vp, lo,
                      J.op[(int)Prec::FP16X2].sigma_t, s));
}

std::vector<int> checked_triples(const Job &J, const int32_t *ijk, int64_t n) {
  if (n < 0 || (n > 0 && !ijk)) throw Fail(TE_EINVAL, "bad triple list");
  for (int64_t t = 0; t < n; ++t) {
    int i = ijk[3 * t], j = ijk[3 * t + 1], k = ijk[3 * t + 2];
    if (i < 0 || i > j || j > k || k >= J.o || (i == j && j == k))
      throw Fail(TE_EINVAL, "triple " + std::to_string(t) + " is not 0<=i<=j<=k<o, not all equal");
  }
  return std::vector<int>(ijk, ijk + 3 * n);
}

void resident_t2_views(const Job &J, const Operands &op, Prec p, WItem &w) {
  const size_t o = J.o, vp2 = (size_t)J.vp * J.vp, es = elem_size(p);
  const int q[3] = {w.i, w.j, w.k};
  for (int x = 0; x < 3; ++x) {
    w.Tc[x] = (const char *)op.T2 + q[x] * vp2 * es;
    w.Tr[x] = (const char *)op.T2 + q[x] * o * vp2 * es;
    w.Tt[x] = op.T2T ? (const char *)op.T2T + q[x] * vp2 * op.lo * es : nullptr;
  }
  w.tcs = o * vp2;
  w.trs = vp2;
  w.tcps = op.tps;
  w.t2tps = op.t2tps;
}

void resident_k_views(const Job &J, int i, int j, int k, EItem &e) {
  const long o = J.o, vp = J.vp;
  const double *K = J.K.as<double>();
  e.Kjk = K + (j * vp * o + k) * vp;
  e.Kik = K + (i * vp * o + k) * vp;
  e.Kij = K + (i * vp * o + j) * vp;
  e.kld = o * vp;
}

void resident_items(const Job &J, const Operands &op, Prec p, int i, int j, int k, int mt,
                    int nt, void *W, double *part, double *out, WItem &w, EItem &e, RItem &r) {
  const size_t vp3 = (size_t)J.vp * J.vp * J.vp, es = elem_size(p);
  w = WItem{};
  w.Xs[0] = (const char *)op.X + (size_t)i * vp3 * es;
  w.Xs[1] = (const char *)op.X + (size_t)j * vp3 * es;
  w.Xs[2] = (const char *)op.X + (size_t)k * vp3 * es;
  w.xps = op.xps;
  w.In = op.In;
  w.ips = op.ips; w.lo = op.lo; w.scale = op.scale;
  w.W = W; w.o = J.o; w.vp = J.vp; w.i = i; w.j = j; w.k = k; w.mt = mt; w.nt = nt;
  resident_t2_views(J, op, p, w);
  e = EItem{};
  resident_k_views(J, i, j, k, e);
  e.W = W; e.t1 = J.t1.as<double>();
  e.eo = J.eo.as<double>(); e.ev = J.ev.as<double>(); e.sext = J.sext.as<int>();
  e.part = part;
  e.part5 = part + J.nsext;
  e.o = J.o; e.v = J.v; e.vp = J.vp; e.nT = J.vp / BOX; e.i = i; e.j = j; e.k = k;
  e.nsext = J.nsext;
  r = RItem{};
  r.part = e.part; r.part5 = e.part5; r.out = out; r.n = J.nsext;
  r.out4 = r.out5 = nullptr;
  r.w = 2.0 - (i == j) - (j == k);
}

// (px|qy) for one occupied pair as a v x v block with row stride vp (Eq. 6
// with two (ov) factors), on stream s.
// The three (ov|ov) blocks of triple (i, j, k) the singles term reads,
// (jb|kc), (ia|kc), (ia|jb) = sum_Q B^Q B^Q (Eq. 6), into dst[0..2] (v x vp
// each), in one launch.
static void assemble_k_blocks(Job &J, int i, int j, int k, double *dst, hipStream_t s) {
  const int o = J.o, v = J.v, vp = J.vp;
  const size_t kblk = (size_t)vp * vp;
  const int pq[3][2] = {{j, k}, {i, k}, {i, j}};
  GemmTN g[3];
  for (int z = 0; z < 3; ++z)
    g[z] = GemmTN{J.Bov + (long)pq[z][0] * v, J.Bov + (long)pq[z][1] * v, dst + z * kblk, v, v,
                  J.naux, (long)o * v, (long)o * v, v, 0, vp, v, 0, 1, 1.0};
  HIPCHK(launch_gemm_tn_batch(g, 3, s));
}

void run_triples(Job &J, Prec p, const int *ijk, long ntr, double *e_sum, double *per_triple,
                 te_stats *st, const SplitOut *split) {
  auto t0 = std::chrono::steady_clock::now();
  const int pslot = (int)p;
  if (J.xc.pslot >= 0 && J.xc.pslot != pslot) {   // slices of another precision
    HIPCHK(hipStreamSynchronize(J.s_main));
    if (J.s_aux) HIPCHK(hipStreamSynchronize(J.s_aux));
    J.xc.release();
  }
  const Operands &op = ensure_prec(J, p);
  const bool fly = !J.x_resident;
  if (!fly && !op.X) throw Fail(TE_EINVAL, "(vv|vo) slices are not resident");

  const int o = J.o, vp = J.vp;
  const WConfig wc = wbuild_config(p, vp);
  const int mt = (int)(((long)vp * vp + wc.bm() - 1) / wc.bm());
  const int nt = (vp + wc.bn() - 1) / wc.bn();
  const int tiles = 3 * mt * nt;
  const int B = batch_size(J, p, ntr);
  const size_t vp3 = (size_t)vp * vp * vp;
  const size_t osz = out_size(p);
  const size_t es = elem_size(p);

  // scratch: W for two batches, partials for two batches, per-triple results,
  // and (on the fly) three (ov|ov) blocks per triple of the two batches
  // (E[4] and E[5] partials per sextet; the two parts per triple when split
  // output is asked for)
  DBuf wbuf, part, eout, e4out, e5out, esum, witems, eitems, ritems, kbuf;
  const size_t kblk = (size_t)vp * vp;
  auto scratch = [&] {
    wbuf.alloc(2 * (size_t)B * 3 * vp3 * osz, &J.used, J.budget);
    part.alloc(2 * (size_t)B * 2 * J.nsext * 8, &J.used, J.budget);
    eout.alloc((size_t)ntr * 8, &J.used, J.budget);
    if (split) {
      e4out.alloc((size_t)ntr * 8, &J.used, J.budget);
      e5out.alloc((size_t)ntr * 8, &J.used, J.budget);
    }
    esum.alloc(3 * 8, &J.used, J.budget);
    if (fly) kbuf.alloc(2 * (size_t)B * 3 * kblk * 8, &J.used, J.budget);
  };
  try {
    scratch();
  } catch (const Fail &f) {
    if (f.s != TE_ENOMEM || !J.xc.mem.p) throw;
    wbuf.release(); part.release(); eout.release(); e4out.release(); e5out.release();
    esum.release(); kbuf.release();
    J.xc.release();                  // a kept cache gives way to this call's scratch
    scratch();
  }

  Plan P;
  size_t slot_bytes = 0;
  // a slot: the (vv|vo) slice, then (host t2) the column panel and the row
  // panel (FP64, FP32) or row form (16-bit parts) of its occupied index
  const size_t vp2 = (size_t)vp * vp;
  const size_t x_bytes = vp3 * es * (size_t)nparts(p);
  const size_t col_bytes = J.t2h ? (size_t)o * vp2 * es * nparts(p) : 0;
  const bool row_form = p != Prec::F64 && p != Prec::F32;   // 16-bit parts, l last
  const size_t row_bytes =
      J.t2h ? (row_form ? vp2 * (size_t)op.lo * es * nparts(p) : (size_t)o * vp2 * es) : 0;
  std::vector<int> after;   // slot contents once this call completes
  if (fly) {
    slot_bytes = x_bytes + col_bytes + row_bytes;
    if (!J.xc.mem.p) {
      if (p != Prec::F64) J.xc.tmp64.alloc(vp3 * 8, &J.used, J.budget);
      if (J.t2h) {
        const size_t pb = (size_t)o * J.v * J.v * 8;
        J.xc.tstg.alloc(pb, &J.used, J.budget);
        for (int x = 0; x < 2; ++x) {
          HIPCHK(hipHostMalloc((void **)&J.xc.pinned[x], pb, hipHostMallocDefault));
          HIPCHK(hipEventCreateWithFlags(&J.xc.pinned_free[x], hipEventDisableTiming));
        }
      }
      long room = (long)((J.budget - std::min(J.budget, J.used + ((size_t)1 << 28))) / slot_bytes);
      int S = J.x_cache ? J.x_cache : (int)std::min<long>(room, o);
      S = std::min(S, o);
      if (S < 3 || S > room) {
        J.xc.release();
        throw Fail(TE_ENOMEM, "no room for three slice-cache slots of " +
                                  std::to_string(slot_bytes) + " bytes in the HBM budget");
      }
      J.xc.mem.alloc((size_t)S * slot_bytes, &J.used, J.budget);
      if (!J.xc.s_fill) HIPCHK(hipStreamCreateWithFlags(&J.xc.s_fill, hipStreamNonBlocking));
      J.xc.S = S;
      J.xc.slot_bytes = slot_bytes;
      J.xc.pslot = pslot;
      J.xc.held.assign(S, -1);
    }
    after = J.xc.held;
    P = plan_on_the_fly(ijk, ntr, B, after);
    J.xc.held.assign(J.xc.S, -1);   // unknown until this call completes
  } else {
    P = plan_resident(ntr, B);
  }
  const long nbatch = (long)P.bfirst.size();

  std::vector<WItem> wi(ntr);
  std::vector<EItem> ei(ntr);
  std::vector<RItem> ri(ntr);
  for (long b = 0; b < nbatch; ++b) {
    for (int q = 0; q < P.bcount[b]; ++q) {
      const long pos = P.bfirst[b] + q, t = P.order[pos];
      const int i = ijk[3 * t], j = ijk[3 * t + 1], k = ijk[3 * t + 2];
      const int sl = (int)(b & 1);
      void *W = wbuf.as<char>() + ((size_t)sl * B + q) * 3 * vp3 * osz;
      WItem &w = wi[pos];
      if (fly) {
        for (int d = 0; d < 3; ++d)
          w.Xs[d] = J.xc.mem.as<char>() + (size_t)P.slot[pos][d] * slot_bytes;
        w.xps = vp3;
      } else {
        w.Xs[0] = (const char *)op.X + (size_t)i * vp3 * es;
        w.Xs[1] = (const char *)op.X + (size_t)j * vp3 * es;
        w.Xs[2] = (const char *)op.X + (size_t)k * vp3 * es;
        w.xps = op.xps;
      }
      w.In = op.In;
      w.ips = op.ips; w.lo = op.lo; w.scale = op.scale;
      w.W = W; w.o = o; w.vp = vp; w.i = i; w.j = j; w.k = k; w.mt = mt; w.nt = nt;
      if (J.t2h) {
        for (int d = 0; d < 3; ++d) {
          const char *sb = J.xc.mem.as<char>() + (size_t)P.slot[pos][d] * slot_bytes;
          w.Tc[d] = sb + x_bytes;
          w.Tr[d] = w.Tt[d] = sb + x_bytes + col_bytes;
        }
        w.tcs = vp2; w.trs = vp2; w.tcps = (size_t)o * vp2; w.t2tps = vp2 * (size_t)op.lo;
      } else {
        resident_t2_views(J, op, p, w);
      }
      EItem &e = ei[pos];
      if (fly) {
        const double *kb = kbuf.as<double>() + ((size_t)sl * B + q) * 3 * kblk;
        e.Kjk = kb; e.Kik = kb + kblk; e.Kij = kb + 2 * kblk; e.kld = vp;
      } else {
        resident_k_views(J, i, j, k, e);
      }
      e.W = W; e.t1 = J.t1.as<double>();
      e.eo = J.eo.as<double>(); e.ev = J.ev.as<double>(); e.sext = J.sext.as<int>();
      e.part = part.as<double>() + ((size_t)sl * B + q) * 2 * J.nsext;
      e.part5 = e.part + J.nsext;
      e.o = o; e.v = J.v; e.vp = vp; e.nT = vp / BOX; e.i = i; e.j = j; e.k = k;
      e.nsext = J.nsext;
      RItem &r = ri[pos];
      r.part = e.part; r.part5 = e.part5; r.out = eout.as<double>() + t; r.n = J.nsext;
      r.out4 = split ? e4out.as<double>() + t : nullptr;
      r.out5 = split ? e5out.as<double>() + t : nullptr;
      r.w = 2.0 - (i == j) - (j == k);
    }
  }
  witems.alloc(ntr * sizeof(WItem), &J.used, J.budget);
  eitems.alloc(ntr * sizeof(EItem), &J.used, J.budget);
  ritems.alloc(ntr * sizeof(RItem), &J.used, J.budget);
  HIPCHK(hipMemcpyAsync(witems.p, wi.data(), ntr * sizeof(WItem), hipMemcpyHostToDevice, J.s_main));
  HIPCHK(hipMemcpyAsync(eitems.p, ei.data(), ntr * sizeof(EItem), hipMemcpyHostToDevice, J.s_main));
  HIPCHK(hipMemcpyAsync(ritems.p, ri.data(), ntr * sizeof(RItem), hipMemcpyHostToDevice, J.s_main));
  // everything before the first launch (operand conversion, scratch and
  // slice-cache allocation, planning, item upload) is set-up, not per triple
  HIPCHK(hipStreamSynchronize(J.s_main));
  auto t1 = std::chrono::steady_clock::now();
  HIPCHK(hipEventRecord(J.ev_start, J.s_main));
  HIPCHK(hipStreamWaitEvent(J.s_aux, J.ev_start, 0));

  const bool f64 = p == Prec::F64;
  // timing events around every launch (device time of each kernel)
  TimingEvents tw(nbatch), te_(nbatch), ta(fly ? nbatch : 0);
  // on-the-fly mode: batch whose W build last read each cache slot (-1:
  // none in this call; earlier calls have completed)
  std::vector<long> last_read(fly ? J.xc.S : 0, -1);
  for (long b = 0; b < nbatch; ++b) {
    const int slot = (int)(b & 1);
    const long first = P.bfirst[b];
    const int cnt = P.bcount[b];
    hipStream_t sw = J.s_aux;
    if (b >= 2) HIPCHK(hipStreamWaitEvent(sw, J.ev_e[slot], 0));
    // slices (and host-t2 panels) this batch needs: filled on the fill
    // stream, each after the last W build that read its slot (the end-of-
    // build timing event of that batch), so that fills run ahead of and
    // beside earlier W builds; this batch's W build waits for them
    if (fly) {
      for (auto &ld : P.loads[b]) {
        const long lr = last_read[ld.second];
        if (lr >= 0) HIPCHK(hipStreamWaitEvent(J.xc.s_fill, tw.stop[lr], 0));
      }
      HIPCHK(hipEventRecord(ta.start[b], J.xc.s_fill));
      for (auto &ld : P.loads[b]) {
        char *sb = J.xc.mem.as<char>() + (size_t)ld.second * slot_bytes;
        assemble_slice(J, p, ld.first, sb, J.xc.tmp64.as<double>(), J.xc.s_fill);
        if (J.t2h)
          fill_panels(J, p, ld.first, sb + x_bytes, sb + x_bytes + col_bytes, J.xc.s_fill);
      }
      HIPCHK(hipEventRecord(ta.stop[b], J.xc.s_fill));
      HIPCHK(hipStreamWaitEvent(sw, ta.stop[b], 0));
    }
    HIPCHK(hipEventRecord(tw.start[b], sw));
    HIPCHK(launch_wbuild(p, witems.as<WItem>() + first, nullptr, cnt, tiles, (long)cnt * tiles,
                         wc, sw));
    HIPCHK(hipEventRecord(tw.stop[b], sw));
    HIPCHK(hipEventRecord(J.ev_w[slot], sw));
    if (fly)   // the slots this batch's W build reads
      for (int q = 0; q < cnt; ++q)
        for (int d = 0; d < 3; ++d) last_read[P.slot[first + q][d]] = b;
    // the batch's (ov|ov) blocks, on the energy stream while W is built (the
    // energy launch two batches back, the last reader of these blocks, is
    // earlier on the same stream)
    if (fly) {
      for (int q = 0; q < cnt; ++q) {
        const long t = P.order[first + q];
        const int i = ijk[3 * t], j = ijk[3 * t + 1], k = ijk[3 * t + 2];
        double *kb = kbuf.as<double>() + ((size_t)slot * B + q) * 3 * kblk;
        assemble_k_blocks(J, i, j, k, kb, J.s_main);
      }
    }
    HIPCHK(hipStreamWaitEvent(J.s_main, J.ev_w[slot], 0));
    HIPCHK(hipEventRecord(te_.start[b], J.s_main));
    HIPCHK(launch_energy(f64, eitems.as<EItem>() + first, nullptr, cnt, J.nsext,
                         (long)cnt * J.nsext, J.s_main));
    HIPCHK(hipEventRecord(te_.stop[b], J.s_main));
    HIPCHK(launch_reduce(ritems.as<RItem>() + first, cnt, J.s_main));
    HIPCHK(hipEventRecord(J.ev_e[slot], J.s_main));
  }
  HIPCHK(launch_sum(eout.as<double>(), ntr, esum.as<double>(), J.s_main));
  if (split) {
    HIPCHK(launch_sum(e4out.as<double>(), ntr, esum.as<double>() + 1, J.s_main));
    HIPCHK(launch_sum(e5out.as<double>(), ntr, esum.as<double>() + 2, J.s_main));
  }
  double Es[3] = {0.0, 0.0, 0.0};
  HIPCHK(hipMemcpyAsync(Es, esum.p, 3 * 8, hipMemcpyDeviceToHost, J.s_main));
  if (per_triple)
    HIPCHK(hipMemcpyAsync(per_triple, eout.p, ntr * 8, hipMemcpyDeviceToHost, J.s_main));
  if (split && split->pt4)
    HIPCHK(hipMemcpyAsync(split->pt4, e4out.p, ntr * 8, hipMemcpyDeviceToHost, J.s_main));
  if (split && split->pt5)
    HIPCHK(hipMemcpyAsync(split->pt5, e5out.p, ntr * 8, hipMemcpyDeviceToHost, J.s_main));
  HIPCHK(hipStreamSynchronize(J.s_main));
  if (fly) J.xc.held = after;
  auto t2 = std::chrono::steady_clock::now();
  const double E = Es[0];
  if (e_sum) *e_sum = E;
  if (split && split->e4_sum) *split->e4_sum = Es[1];
  if (split && split->e5_sum) *split->e5_sum = Es[2];
  if (st) {
    st->seconds = std::chrono::duration<double>(t2 - t0).count();
    st->stage_seconds = std::chrono::duration<double>(t1 - t0).count();
    st->n_triples = ntr;
    st->flops = (double)ntr * flops_per_triple(o, J.v);
    st->tflops = st->flops / std::max(st->seconds, 1e-12) / 1e12;
    st->assemble_flops = (double)P.nloads * 2.0 * J.naux * (double)J.v * J.v * J.v
                       + (fly ? (double)ntr * 3 * 2.0 * J.naux * (double)J.v * J.v : 0.0);
    st->w_kernel_seconds = tw.total();
    st->w_launches = nbatch;
    st->e_kernel_seconds = te_.total();
    st->e_launches = nbatch;
    st->slices_assembled = P.nloads;
    st->assemble_seconds = fly ? ta.total() : 0.0;
    st->cache_slices = fly ? J.xc.S : 0;
  }
}

int64_t plan_slice_loads(int o, int S, int B) {
  std::vector<int> t = triple_list_host(o);
  std::vector<int> held(S, -1);
  Plan P = plan_on_the_fly(t.data(), (long)t.size() / 3, B, held);
  return P.nloads;
}

Job::~Job() {
  if (dev_set) (void)hipSetDevice(device);
  if (s_main) (void)hipStreamSynchronize(s_main);
  if (s_aux) {
    (void)hipStreamSynchronize(s_aux);
    (void)hipStreamDestroy(s_aux);
  }
  for (int q = 0; q < 2; ++q) {
    if (ev_w[q]) (void)hipEventDestroy(ev_w[q]);
    if (ev_e[q]) (void)hipEventDestroy(ev_e[q]);
  }
  if (ev_start) (void)hipEventDestroy(ev_start);
  if (own_main && s_main) (void)hipStreamDestroy(s_main);
  xc.release();
  if (xc.s_fill) (void)hipStreamDestroy(xc.s_fill);
}

void Job::SliceCache::release() {
  if (s_fill) (void)hipStreamSynchronize(s_fill);   // fills in flight finish first
  mem.release();
  tmp64.release();
  tstg.release();
  held.clear();
  S = 0;
  pslot = -1;
  for (int x = 0; x < 2; ++x) {
    if (pinned_free[x]) {
      (void)hipEventSynchronize(pinned_free[x]);
      (void)hipEventDestroy(pinned_free[x]);
      pinned_free[x] = nullptr;
    }
    if (pinned[x]) {
      (void)hipHostFree(pinned[x]);
      pinned[x] = nullptr;
    }
  }
  nfill = 0;
}

static void check_problem(const te_problem *P) {
  if (!P) throw Fail(TE_EINVAL, "problem is NULL");
  if (P->o < 1 || P->v < 1 || P->naux < 0)
    throw Fail(TE_EINVAL, "need o >= 1, v >= 1, naux >= 0");
  if (pad_v(P->v) / BOX > 1023) throw Fail(TE_EINVAL, "v above 8184 is not supported");
  if (P->mem != TE_MEM_HOST && P->mem != TE_MEM_DEVICE) throw Fail(TE_EINVAL, "bad memory kind");
  if (!P->eps_occ || !P->eps_vir || !P->t1 || !P->t2)
    throw Fail(TE_EINVAL, "eps_occ, eps_vir, t1 and t2 are required");
  if (P->naux > 0 && (!P->B_oo || !P->B_ov || !P->B_vv))
    throw Fail(TE_EINVAL, "naux > 0 needs B_oo, B_ov and B_vv");
  if (P->naux == 0 && (!P->ovvv || !P->ovoo || !P->ovov))
    throw Fail(TE_EINVAL, "naux == 0 needs ovvv, ovoo and ovov");
}

static void check_host_values(const te_problem &P) {
  if (P.mem != TE_MEM_HOST) return;
  auto finite = [](const double *x, size_t n) {
    for (size_t q = 0; q < n; ++q)
      if (!std::isfinite(x[q])) return false;
    return true;
  };
  const size_t o = P.o, v = P.v;
  if (!finite(P.eps_occ, o) || !finite(P.eps_vir, v) || !finite(P.t1, o * v))
    throw Fail(TE_EINVAL, "input holds a non-finite value");
}

// Host t2 (left in host memory): finite values and t_ij^ab = t_ji^ba, the
// checks the device makes on a staged t2.
static void check_host_t2(const te_problem &P) {
  const size_t o = P.o, v = P.v, v2 = v * v;
  double amax = 0.0, dmax = 0.0;
  for (size_t i = 0; i < o; ++i)
    for (size_t j = 0; j < o; ++j)
      for (size_t a = 0; a < v; ++a)
        for (size_t b = 0; b < v; ++b) {
          const double x = P.t2[(i * o + j) * v2 + a * v + b];
          if (!std::isfinite(x)) throw Fail(TE_EINVAL, "input holds a non-finite value");
          amax = std::max(amax, std::abs(x));
          dmax = std::max(dmax, std::abs(x - P.t2[(j * o + i) * v2 + b * v + a]));
        }
  if (dmax > 1e-12 * std::max(amax, 1e-300))
    throw Fail(TE_EINVAL, "t2 is not pair-symmetric: max |t_ij^ab - t_ji^ba| = " +
                              std::to_string(dmax));
}

int out_bytes(Prec p) { return p == Prec::F64 ? 8 : 4; }

size_t job_footprint(int o, int v, int naux, Prec p) {
  const size_t O = o, V = v, VP = pad_v(v), N = naux;
  const size_t nT = VP / BOX, nsext = nT * (nT + 1) * (nT + 2) / 6;
  const size_t nt = (size_t)te_num_triples(o);
  size_t b = 8 * (O + VP + O * VP) + 8 * O * O * VP * VP * 2 + 8 * O * VP * O * O;
  b += 4 * nsext + 8 * nt + 8;
  // staging temporaries: unpadded host copies and the factors
  b += 8 * (O + V + O * V + O * O * V * V);
  b += naux > 0 ? 8 * N * (O * V + O * O + V * V) : 8 * (O * V * V * V + O * V * O * O + O * V * O * V);
  const size_t nX = O * VP * VP * VP, nT2 = O * O * VP * VP, nIn = O * VP * O * O;
  b += 8 * nX;
  if (p == Prec::F32) b += 4 * (nX + nT2 + nIn);
  if (p == Prec::BF16X3 || p == Prec::BF16X2 || p == Prec::FP16X2) {
    const size_t LO = (O + 7) / 8 * 8;
    b += (p == Prec::BF16X3 ? 6 : 4) * (nX + nT2 + O * VP * O * LO + O * VP * VP * LO);
  }
  return b + 32 * 256;
}

Job *make_job(const te_problem *P, const te_config *cfg_in, const JobOpts *opts) {
  check_problem(P);
  te_config cfg{};
  if (cfg_in) cfg = *cfg_in;
  if (cfg.x_mode < TE_X_AUTO || cfg.x_mode > TE_X_ON_THE_FLY)
    throw Fail(TE_EINVAL, "bad x_mode");
  if (cfg.t2_host) {
    if (P->naux == 0) throw Fail(TE_EINVAL, "t2 in host memory needs the factors (naux > 0)");
    if (P->mem != TE_MEM_HOST) throw Fail(TE_EINVAL, "t2 in host memory needs host arrays");
    if (cfg.x_mode == TE_X_RESIDENT)
      throw Fail(TE_EINVAL, "t2 in host memory implies on-the-fly (vv|vo) slices");
    if (opts) throw Fail(TE_EINVAL, "server jobs keep t2 on the device");
  }
  if (cfg.validate) check_host_values(*P);
  if (cfg.validate && cfg.t2_host) check_host_t2(*P);
  int ndev = 0;
  HIPCHK(hipGetDeviceCount(&ndev));
  if (cfg.device < 0 || cfg.device >= ndev) throw Fail(TE_EINVAL, "bad device ordinal");
  HIPCHK(hipSetDevice(cfg.device));

  std::unique_ptr<Job> J(new Job());
  J->device = cfg.device;
  J->dev_set = true;
  J->o = P->o; J->v = P->v; J->vp = pad_v(P->v); J->naux = P->naux; J->mem = P->mem;
  if (opts && opts->arena) J->arena = opts->arena;
  if (opts && opts->budget) {
    J->budget = opts->budget;
  } else if (cfg.hbm_budget) {
    J->budget = cfg.hbm_budget;
  } else {
    size_t freeb = 0, total = 0;
    HIPCHK(hipMemGetInfo(&freeb, &total));
    J->budget = (size_t)(0.9 * (double)freeb);
  }
  if (opts && opts->stream) {
    J->s_main = opts->stream;
    J->own_main = false;
    J->own_aux = false;
  } else if (cfg.stream) {
    J->s_main = (hipStream_t)cfg.stream;
    J->own_main = false;
  } else {
    HIPCHK(hipStreamCreateWithFlags(&J->s_main, hipStreamNonBlocking));
    J->own_main = true;
  }
  if (J->own_aux) {
    HIPCHK(hipStreamCreateWithFlags(&J->s_aux, hipStreamNonBlocking));
    for (int q = 0; q < 2; ++q) {
      HIPCHK(hipEventCreateWithFlags(&J->ev_w[q], hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&J->ev_e[q], hipEventDisableTiming));
    }
    HIPCHK(hipEventCreateWithFlags(&J->ev_start, hipEventDisableTiming));
  }

  const size_t o = J->o, vp = J->vp;
  const size_t xbytes = o * vp * vp * vp * 8;
  if (cfg.t2_host) J->t2h = P->t2;
  if (P->naux == 0) {
    J->x_resident = true;
  } else if (cfg.t2_host) {
    J->x_resident = false;
  } else if (cfg.x_mode == TE_X_RESIDENT) {
    J->x_resident = true;
  } else if (cfg.x_mode == TE_X_ON_THE_FLY) {
    J->x_resident = false;
  } else {
    J->x_resident = xbytes <= J->budget / 2;
  }
  J->x_cache = std::max(0, cfg.x_cache_slices);

  // sextets of 8^3 boxes
  J->nT = (int)(vp / BOX);
  std::vector<int> sx = sextet_list(J->nT);
  J->nsext = (int)sx.size();
  jalloc(*J, J->sext, sx.size() * sizeof(int));
  HIPCHK(hipMemcpyAsync(J->sext.p, sx.data(), sx.size() * sizeof(int), hipMemcpyHostToDevice,
                        J->s_main));
  HIPCHK(hipStreamSynchronize(J->s_main));

  stage(*J, *P);
  if (cfg.validate) validate_device(*J, *P);
  if (opts) {
    ensure_prec(*J, opts->prec);
    if (opts->drop_fp64_x && opts->prec != Prec::F64) {
      J->X.release();
      J->op[(int)Prec::F64].ready = false;
    }
  }
  return J.release();
}

}  // namespace te

using namespace te;

// ------------------------------------------------------------ C ABI
extern "C" {

te_status te_init(const te_problem *prob, const te_config *cfg, te_job *out) {
  TE_GUARD_BEGIN
  if (!out) return set_error(TE_EINVAL, "out is NULL");
  Job *J = make_job(prob, cfg);
  *out = reinterpret_cast<te_job>(J);
  return TE_OK;
  TE_GUARD_END
}

te_status te_energy(te_job job, te_precision prec, double *e_t, double *per_triple,
                    te_stats *st) {
  TE_GUARD_BEGIN
  if (!job) return set_error(TE_EINVAL, "job is NULL");
  Job &J = *reinterpret_cast<Job *>(job);
  Prec p = to_prec(prec);
  HIPCHK(hipSetDevice(J.device));
  std::vector<int> t = triple_list_host(J.o);
  long n = (long)t.size() / 3;
  double E = 0.0;
  te_stats s{};
  if (n > 0) {
    run_triples(J, p, t.data(), n, &E, per_triple, &s);
  }
  if (e_t) *e_t = E;
  if (st) *st = s;
  return TE_OK;
  TE_GUARD_END
}

te_status te_energy_triples(te_job job, te_precision prec, const int32_t *ijk, int64_t n,
                            double *e_sum, double *per_triple, te_stats *st) {
  TE_GUARD_BEGIN
  if (!job) return set_error(TE_EINVAL, "job is NULL");
  Job &J = *reinterpret_cast<Job *>(job);
  Prec p = to_prec(prec);
  std::vector<int> t = checked_triples(J, ijk, n);
  HIPCHK(hipSetDevice(J.device));
  double E = 0.0;
  te_stats s{};
  if (n > 0) run_triples(J, p, t.data(), (long)n, &E, per_triple, &s);
  if (e_sum) *e_sum = E;
  if (st) *st = s;
  return TE_OK;
  TE_GUARD_END
}

te_status te_energy_terms(te_job job, te_precision prec, const int32_t *ijk, int64_t n,
                          double *e4_sum, double *e5_sum, double *e4, double *e5,
                          te_stats *st) {
  TE_GUARD_BEGIN
  if (!job) return set_error(TE_EINVAL, "job is NULL");
  Job &J = *reinterpret_cast<Job *>(job);
  Prec p = to_prec(prec);
  std::vector<int> t = ijk ? checked_triples(J, ijk, n) : triple_list_host(J.o);
  const long nt = (long)t.size() / 3;
  HIPCHK(hipSetDevice(J.device));
  SplitOut so;
  double E4 = 0.0, E5 = 0.0;
  so.e4_sum = &E4; so.e5_sum = &E5; so.pt4 = e4; so.pt5 = e5;
  te_stats s{};
  if (nt > 0) run_triples(J, p, t.data(), nt, nullptr, nullptr, &s, &so);
  if (e4_sum) *e4_sum = E4;
  if (e5_sum) *e5_sum = E5;
  if (st) *st = s;
  return TE_OK;
  TE_GUARD_END
}

te_status te_free(te_job job) {
  TE_GUARD_BEGIN
  if (!job) return set_error(TE_EINVAL, "job is NULL");
  delete reinterpret_cast<Job *>(job);
  return TE_OK;
  TE_GUARD_END
}

int64_t te_num_triples(int32_t o) {
  if (o < 1) return 0;
  return (int64_t)o * (o + 1) * (o + 2) / 6 - o;
}

te_status te_triple_list(int32_t o, int32_t *ijk) {
  if (o < 1 || !ijk) return set_error(TE_EINVAL, "need o >= 1 and a buffer");
  std::vector<int> t = triple_list_host(o);
  std::memcpy(ijk, t.data(), t.size() * sizeof(int));
  return TE_OK;
}

double te_flops_per_triple(int32_t o, int32_t v) { return flops_per_triple(o, v); }

int64_t te_plan_slice_loads(int32_t o, int32_t cache_slices, int32_t batch) {
  if (o < 1 || cache_slices < 3 || batch < 1) return -1;
  try {
    return plan_slice_loads(o, cache_slices, batch);
  } catch (...) {
    return -1;
  }
}

te_status te_mfma_sustained(int device, te_precision prec, double seconds, double *tflops) {
  TE_GUARD_BEGIN
  if (!tflops || !(seconds > 0.0) || seconds > 60.0)
    return set_error(TE_EINVAL, "need a result pointer and 0 < seconds <= 60");
  Prec p = to_prec(prec);
  int ndev = 0;
  HIPCHK(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return set_error(TE_EINVAL, "bad device ordinal");
  HIPCHK(hipSetDevice(device));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, device));
  const int blocks = 8 * prop.multiProcessorCount;   // 8 waves per SIMD
  DBuf out;
  out.alloc((size_t)blocks * 256 * 8, nullptr, 0);
  hipStream_t s;
  HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  double fl = 0, rate = 0;
  int iters = 256;
  float ms = 0.f;
  for (int rep = 0; rep < 8; ++rep) {     // grow the loop until it runs `seconds`
    HIPCHK(hipEventRecord(e0, s));
    HIPCHK(launch_mfma_probe(p, out.p, blocks, iters, s, &fl));
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    rate = fl / (ms * 1e-3) / 1e12;
    if (ms * 1e-3 >= 0.5 * seconds) break;
    iters = (int)std::min(1e8, iters * std::max(2.0, seconds / std::max(ms * 1e-3, 1e-4)));
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamDestroy(s);
  *tflops = rate;
  return TE_OK;
  TE_GUARD_END
}

const char *te_strerror(te_status s) {
  switch (s) {
    case TE_OK: return "ok";
    case TE_PENDING: return "pending";
    case TE_EINVAL: return "invalid argument";
    case TE_ENOMEM: return "does not fit the HBM budget";
    case TE_EDEVICE: return "HIP runtime error";
    case TE_EBUSY: return "busy";
    case TE_ENOTFOUND: return "unknown ticket";
    case TE_ECANCELED: return "canceled";
    case TE_EIO: return "checkpoint file I/O failed";
  }
  return "unknown status";
}

const char *te_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
