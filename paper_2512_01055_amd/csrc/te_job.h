// Host-side job state shared by the C-ABI entry points and the server.
#pragma once
#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "te.h"
#include "te_internal.h"

namespace te {

struct Fail {
  te_status s;
  std::string msg;
  Fail(te_status s_, std::string m);
};

void hip_check(hipError_t e, const char *what, int line);
#define HIPCHK(call) ::te::hip_check((call), #call, __LINE__)

te_status set_error(te_status s, const std::string &m);

// Body of every C-ABI entry point: exceptions become status codes.
#define TE_GUARD_BEGIN try {
#define TE_GUARD_END                                                                        \
  }                                                                                         \
  catch (const ::te::Fail &f) { return ::te::set_error(f.s, f.msg); }                       \
  catch (const std::bad_alloc &) { return ::te::set_error(TE_ENOMEM, "host allocation failed"); } \
  catch (...) { return ::te::set_error(TE_EDEVICE, "unexpected exception"); }

inline Prec to_prec(te_precision p) {
  if (p < TE_FP64 || p > TE_FP16X2) throw Fail(TE_EINVAL, "bad precision");
  return static_cast<Prec>(p);
}

// One device allocation carved up on the host: first fit over a free list,
// 256-byte granules. Freeing never touches the device, so a server can
// recycle memory of finished jobs while other work is in flight (it frees a
// range only after the work that used it has completed).
struct Arena {
  char *base = nullptr;
  size_t cap = 0, used = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  std::mutex mu;
  void init(size_t bytes);          // one hipMalloc of the whole budget
  void destroy();
  void *take(size_t n);              // nullptr when no free range fits
  void give(void *p, size_t n);
  size_t largest_free();
};

// Device allocation charged against a job's HBM budget (from an arena when
// one is given, else straight from hipMalloc).
struct DBuf {
  void *p = nullptr;
  size_t bytes = 0;
  size_t *acct = nullptr;
  Arena *arena = nullptr;
  DBuf() = default;
  DBuf(const DBuf &) = delete;
  DBuf &operator=(const DBuf &) = delete;
  ~DBuf();
  void alloc(size_t n, size_t *account, size_t budget, Arena *ar = nullptr);
  void release();
  template <typename T> T *as() const { return reinterpret_cast<T *>(p); }
};

// Operand copies of one precision (FP64 points at the staged arrays).
struct Operands {
  bool ready = false;
  const void *X = nullptr, *T2 = nullptr, *In = nullptr, *T2T = nullptr;
  size_t xps = 0, tps = 0, ips = 0, t2tps = 0;
  int lo = 0;     // occupied row length of In / T2T
  float scale = 1.0f;  // FP16 parts: 1 / (sigma_X sigma_T); 1 otherwise
  double sigma_x = 1.0, sigma_t = 1.0;
  DBuf X_own, T2_own, In_own, T2T_own;
};

struct Job {
  int o = 0, v = 0, vp = 0, naux = 0, device = 0;
  te_memkind mem = TE_MEM_HOST;
  bool dev_set = false;
  hipStream_t s_main = nullptr, s_aux = nullptr;   // energy and copies; W builds
  bool own_main = false;
  hipEvent_t ev_w[2] = {nullptr, nullptr}, ev_e[2] = {nullptr, nullptr}, ev_start = nullptr;
  size_t budget = 0, used = 0;
  bool x_resident = true;
  int x_cache = 0;             // on-the-fly mode: slices cached (0: automatic)
  Arena *arena = nullptr;      // server jobs allocate from the server's arena
  bool own_aux = true;         // false: no second stream / events (server jobs)

  DBuf eo, ev, t1, K, In, X, t2_own, sext;
  const double *t2 = nullptr;      // device t2 (padded), or null with t2 in host memory
  const double *t2h = nullptr;     // host t2 [o][o][v][v] when it stays in host memory
  DBuf Bov_own, Boo_own, Bvv_own;
  const double *Bov = nullptr, *Boo = nullptr, *Bvv = nullptr;
  // max |(px|yf)| bound from the factors, max_px |B_px| max_yf |B_yf| (set
  // at staging, while the factors are present; 0 with explicit integrals)
  double x_bound = 0.0;
  Operands op[5];
  // On-the-fly mode: the (vv|vo) slice cache and which occupied index each
  // slot holds (-1: empty), kept across calls in one precision so that a job
  // evaluated in pieces does not start from a cold cache.
  struct SliceCache {
    int pslot = -1;               // operand slot (precision) of the slices
    int S = 0;
    size_t slot_bytes = 0;
    DBuf mem, tmp64;
    std::vector<int> held;
    // host t2: FP64 column panel on the device, two pinned host bounce
    // buffers used in turn, and the events after which each may be refilled
    DBuf tstg;
    double *pinned[2] = {nullptr, nullptr};
    hipEvent_t pinned_free[2] = {nullptr, nullptr};
    int nfill = 0;                // panel fills so far (selects the bounce buffer)
    // stream the slices and panels are filled on, ahead of the W builds:
    // a fill waits only for the last W build that read its slot
    hipStream_t s_fill = nullptr;
    void release();
  } xc;
  int nT = 0, nsext = 0;
  ~Job();
};

// Optional knobs for jobs created by the server.
struct JobOpts {
  Arena *arena = nullptr;
  hipStream_t stream = nullptr;   // staging stream (not owned)
  size_t budget = 0;              // 0: from te_config / free memory
  bool drop_fp64_x = false;       // free the FP64 (vv|vo) copy after converting
  Prec prec = Prec::F64;          // precision staged eagerly
};

Job *make_job(const te_problem *P, const te_config *cfg, const JobOpts *opts = nullptr);
void jalloc(Job &J, DBuf &b, size_t n);
size_t job_footprint(int o, int v, int naux, Prec p);
int out_bytes(Prec p);
const Operands &ensure_prec(Job &J, Prec p);
void resident_k_views(const Job &J, int i, int j, int k, EItem &e);
// t2 views of a W item over the device-resident t2 (and row form) of `op`;
// w.i, w.j, w.k must be set.
void resident_t2_views(const Job &J, const Operands &op, Prec p, WItem &w);
// The three launch items of triple (i, j, k) of a job whose (vv|vo) slices
// and (ov|ov) array are resident: W build (W: its three boxed shares), energy
// (part: 2 nsext sextet partials, E[4] then E[5]) and reduction (out: the
// weighted per-triple result). mt, nt: tiles of the W build along M and N.
void resident_items(const Job &J, const Operands &op, Prec p, int i, int j, int k, int mt,
                    int nt, void *W, double *part, double *out, WItem &w, EItem &e, RItem &r);
// Optional E[4] / E[5] outputs of run_triples (any pointer may be null).
struct SplitOut {
  double *e4_sum = nullptr, *e5_sum = nullptr;   // sums over the listed triples
  double *pt4 = nullptr, *pt5 = nullptr;         // host [ntr] per-triple parts
};
void run_triples(Job &J, Prec p, const int *ijk, long ntr, double *e_sum, double *per_triple,
                 te_stats *st, const SplitOut *split = nullptr);
std::vector<int> triple_list_host(int o);
// Copy of a caller's [n][3] triple list after checking 0 <= i <= j <= k < o,
// not all equal (TE_EINVAL otherwise).
std::vector<int> checked_triples(const Job &J, const int32_t *ijk, int64_t n);
std::vector<int> sextet_list(int nT);
double flops_per_triple(int o, int v);
int64_t plan_slice_loads(int o, int S, int B);

}  // namespace te
