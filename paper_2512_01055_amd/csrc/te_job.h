// Host-side job state shared by the C-ABI entry points and the server.
#pragma once
#include <hip/hip_runtime.h>

#include <memory>
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

// Device allocation charged against a job's HBM budget.
struct DBuf {
  void *p = nullptr;
  size_t bytes = 0;
  size_t *acct = nullptr;
  DBuf() = default;
  DBuf(const DBuf &) = delete;
  DBuf &operator=(const DBuf &) = delete;
  ~DBuf();
  void alloc(size_t n, size_t *account, size_t budget);
  void release();
  template <typename T> T *as() const { return reinterpret_cast<T *>(p); }
};

// Operand copies of one precision (FP64 points at the staged arrays).
struct Operands {
  bool ready = false;
  const void *X = nullptr, *T2 = nullptr, *In = nullptr;
  size_t xps = 0, tps = 0, ips = 0;
  DBuf X_own, T2_own, In_own;
};

struct Job {
  int o = 0, v = 0, vp = 0, naux = 0, device = 0;
  te_memkind mem = TE_MEM_HOST;
  bool dev_set = false;
  hipStream_t s_main = nullptr, s_aux = nullptr;
  bool own_main = false;
  hipEvent_t ev_w[2] = {nullptr, nullptr}, ev_e[2] = {nullptr, nullptr}, ev_start = nullptr;
  size_t budget = 0, used = 0;
  bool x_resident = true;

  DBuf eo, ev, t1, K, In, X, t2_own, sext;
  const double *t2 = nullptr;
  DBuf Bov_own, Boo_own, Bvv_own;
  const double *Bov = nullptr, *Boo = nullptr, *Bvv = nullptr;
  Operands op[4];
  int nT = 0, nsext = 0;
  ~Job();
};

Job *make_job(const te_problem *P, const te_config *cfg);
const Operands &ensure_prec(Job &J, Prec p);
void run_triples(Job &J, Prec p, const int *ijk, long ntr, double *e_sum, double *per_triple,
                 te_stats *st);
std::vector<int> triple_list_host(int o);
std::vector<int> sextet_list(int nT);
double flops_per_triple(int o, int v);

}  // namespace te
