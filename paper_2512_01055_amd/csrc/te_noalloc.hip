// te_energy_triples_noalloc: te_energy_triples for callers that cannot
// allocate device memory. Every per-call device buffer of the triples
// evaluation -- the launch items, the W shares of the batches in flight, the
// per-sextet partials, the per-triple results and their sum -- is carved out
// of one file-scope device array instead of being allocated. The kernels are
// the ones te_energy_triples launches, with the same items, so the results
// are bitwise the same.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <string>
#include <vector>

#include "te_job.h"

namespace te {
namespace {

constexpr size_t kScratchBytes = (size_t)512 << 20;

// One copy per device, held until the process ends. Host code never uses
// this name as an address: it reads the device address once per device
// with hipGetSymbolAddress and passes that on.
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;                       // guards g_ptr and g_dev_mu creation
char *g_ptr[kMaxDevices] = {};         // device address of `scratch` per device
std::mutex g_dev_mu[kMaxDevices];      // one call at a time per device in this process

// Device address of this device's array (the device must be current).
char *scratch_ptr(int dev) {
  if (dev < 0 || dev >= kMaxDevices) throw Fail(TE_EINVAL, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      throw Fail(TE_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                 hipGetErrorString(e));
    g_ptr[dev] = static_cast<char *>(p);
  }
  return g_ptr[dev];
}

size_t up256(size_t n) { return (n + 255) & ~(size_t)255; }

// Bump allocation inside the array; throws when the call needs more than it
// holds.
struct Carve {
  char *base;
  size_t off = 0;
  Carve(char *b) : base(b) {}
  char *take(size_t n) {
    char *p = base + off;
    off += up256(n);
    return p;
  }
};

}  // namespace

static void run_noalloc(Job &J, Prec p, const int *ijk, long ntr, double *e_sum,
                        double *per_triple, te_stats *st) {
  auto t0 = std::chrono::steady_clock::now();
  if (!J.x_resident || J.t2h)
    throw Fail(TE_EINVAL, "the no-allocation path needs resident (vv|vo) slices and device t2");
  if (!J.s_aux) throw Fail(TE_EINVAL, "the no-allocation path needs a job from te_init");
  // FP64 operands are views of the staged arrays (setting them up allocates
  // nothing); a reduced-precision copy must exist already
  if (p != Prec::F64 && !J.op[(int)p].ready)
    throw Fail(TE_EINVAL, "no operand copy in this precision: evaluate once with "
                          "te_energy_triples in it first (that call converts the operands)");
  const Operands &op = ensure_prec(J, p);
  const int o = J.o, vp = J.vp;
  const WConfig wc = wbuild_config(p, vp);
  const int mt = (int)(((long)vp * vp + wc.bm() - 1) / wc.bm());
  const int nt = (vp + wc.bn() - 1) / wc.bn();
  const int tiles = 3 * mt * nt;
  const size_t vp3 = (size_t)vp * vp * vp;
  const size_t osz = (size_t)out_bytes(p);

  // layout: items and per-triple results for the whole list, then per batch
  // slot the W shares and the sextet partials of up to B triples
  const size_t fixed = up256(ntr * sizeof(WItem)) + up256(ntr * sizeof(EItem)) +
                       up256(ntr * sizeof(RItem)) + up256(ntr * 8) + up256(8);
  const size_t per_triple_bytes = up256(3 * vp3 * osz) + up256(2 * (size_t)J.nsext * 8);
  if (fixed + per_triple_bytes > kScratchBytes)
    throw Fail(TE_EINVAL, "problem too large for the no-allocation path: one triple needs " +
                              std::to_string(fixed + per_triple_bytes) + " bytes of the " +
                              std::to_string(kScratchBytes) + "-byte static scratch");
  const long cap = (long)((kScratchBytes - fixed) / per_triple_bytes);   // triples resident
  const int nslot = cap >= 2 ? 2 : 1;
  // triples per launch: at least 16k workgroup tiles (a few waves of
  // workgroups over the chip), within the scratch
  long B = std::max(1L, (16384L + tiles - 1) / tiles);
  B = std::min(B, std::max(1L, cap / nslot));
  B = std::min(B, ntr);

  char *base = scratch_ptr(J.device);
  Carve cv(base);
  WItem *d_wi = reinterpret_cast<WItem *>(cv.take(ntr * sizeof(WItem)));
  EItem *d_ei = reinterpret_cast<EItem *>(cv.take(ntr * sizeof(EItem)));
  RItem *d_ri = reinterpret_cast<RItem *>(cv.take(ntr * sizeof(RItem)));
  double *d_out = reinterpret_cast<double *>(cv.take(ntr * 8));
  double *d_sum = reinterpret_cast<double *>(cv.take(8));
  char *wslot[2] = {nullptr, nullptr};
  double *pslot[2] = {nullptr, nullptr};
  for (int s = 0; s < nslot; ++s) {
    wslot[s] = cv.take(B * up256(3 * vp3 * osz));
    pslot[s] = reinterpret_cast<double *>(cv.take(B * up256(2 * (size_t)J.nsext * 8)));
  }
  if (cv.off > kScratchBytes) throw Fail(TE_EDEVICE, "scratch layout overflow");

  // launch items (every output the kernels write is overwritten in full, so
  // nothing in the array has to start at zero)
  std::vector<WItem> wi(ntr);
  std::vector<EItem> ei(ntr);
  std::vector<RItem> ri(ntr);
  const long nbatch = (ntr + B - 1) / B;
  for (long b = 0; b < nbatch; ++b) {
    const int s = (int)(b % nslot);
    for (long q = 0; q < B && b * B + q < ntr; ++q) {
      const long t = b * B + q;
      void *W = wslot[s] + q * up256(3 * vp3 * osz);
      double *part = pslot[s] + q * (up256(2 * (size_t)J.nsext * 8) / 8);
      resident_items(J, op, p, ijk[3 * t], ijk[3 * t + 1], ijk[3 * t + 2], mt, nt, W, part,
                     d_out + t, wi[t], ei[t], ri[t]);
    }
  }
  HIPCHK(hipMemcpyAsync(d_wi, wi.data(), ntr * sizeof(WItem), hipMemcpyHostToDevice, J.s_main));
  HIPCHK(hipMemcpyAsync(d_ei, ei.data(), ntr * sizeof(EItem), hipMemcpyHostToDevice, J.s_main));
  HIPCHK(hipMemcpyAsync(d_ri, ri.data(), ntr * sizeof(RItem), hipMemcpyHostToDevice, J.s_main));
  HIPCHK(hipEventRecord(J.ev_start, J.s_main));
  HIPCHK(hipStreamWaitEvent(J.s_aux, J.ev_start, 0));

  // W builds on the second stream, energy and reduction on the first; a
  // batch slot is refilled only after the energy launch that read it
  const bool f64 = p == Prec::F64;
  for (long b = 0; b < nbatch; ++b) {
    const int s = (int)(b % nslot);
    const long first = b * B;
    const int cnt = (int)std::min<long>(B, ntr - first);
    if (b >= nslot) HIPCHK(hipStreamWaitEvent(J.s_aux, J.ev_e[s], 0));
    HIPCHK(launch_wbuild(p, d_wi + first, nullptr, cnt, tiles, (long)cnt * tiles, wc, J.s_aux));
    HIPCHK(hipEventRecord(J.ev_w[s], J.s_aux));
    HIPCHK(hipStreamWaitEvent(J.s_main, J.ev_w[s], 0));
    HIPCHK(launch_energy(f64, d_ei + first, nullptr, cnt, J.nsext, (long)cnt * J.nsext,
                         J.s_main));
    HIPCHK(launch_reduce(d_ri + first, cnt, J.s_main));
    HIPCHK(hipEventRecord(J.ev_e[s], J.s_main));
  }
  HIPCHK(launch_sum(d_out, ntr, d_sum, J.s_main));
  double E = 0.0;
  HIPCHK(hipMemcpyAsync(&E, d_sum, 8, hipMemcpyDeviceToHost, J.s_main));
  if (per_triple)
    HIPCHK(hipMemcpyAsync(per_triple, d_out, ntr * 8, hipMemcpyDeviceToHost, J.s_main));
  HIPCHK(hipStreamSynchronize(J.s_main));
  auto t1 = std::chrono::steady_clock::now();
  if (e_sum) *e_sum = E;
  if (st) {
    *st = te_stats{};
    st->seconds = std::chrono::duration<double>(t1 - t0).count();
    st->n_triples = ntr;
    st->flops = (double)ntr * flops_per_triple(o, J.v);
    st->tflops = st->flops / std::max(st->seconds, 1e-12) / 1e12;
  }
}

}  // namespace te

using namespace te;

extern "C" te_status te_energy_triples_noalloc(te_job job, te_precision prec,
                                               const int32_t *ijk, int64_t n, double *e_sum,
                                               double *per_triple, te_stats *st) {
  TE_GUARD_BEGIN
  if (!job) return set_error(TE_EINVAL, "job is NULL");
  Job &J = *reinterpret_cast<Job *>(job);
  Prec p = to_prec(prec);
  std::vector<int> t = checked_triples(J, ijk, n);
  HIPCHK(hipSetDevice(J.device));
  if (J.device < 0 || J.device >= kMaxDevices) return set_error(TE_EINVAL, "device ordinal out of range");
  std::lock_guard<std::mutex> lk(g_dev_mu[J.device]);
  double E = 0.0;
  te_stats s{};
  if (n > 0) run_noalloc(J, p, t.data(), (long)n, &E, per_triple, &s);
  if (e_sum) *e_sum = E;
  if (st) *st = s;
  return TE_OK;
  TE_GUARD_END
}
