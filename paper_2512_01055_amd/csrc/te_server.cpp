// Continuous-batching (T) server.
//
// Jobs of mixed (o, v) are queued by te_submit, admitted when their HBM
// footprint fits a server-wide arena, staged by a staging thread (integral
// assembly and precision copies on their own stream, overlapping the compute
// of resident jobs), and their occupied triples are packed with those of every
// other resident job of the same precision into shared launches (small jobs
// first, then large ones in admission order): one W-build launch per tile shape and one
// energy launch per round, mapping tiles and sextet blocks to (job, triple)
// items. Three rounds are in flight at once (three scratch slots).
// A job finishes with a fixed-order sum of its per-triple partials, so its
// result is bitwise the one te_energy computes for it alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "te.h"
#include "te_internal.h"
#include "te_job.h"

namespace te {
namespace {

using clk = std::chrono::steady_clock;

// Host copy of a submitted problem (te_submit returns before staging), or
// the caller's pointers when the server borrows its inputs.
struct HostCopy {
  te_problem p{};
  std::vector<double> a[10];
  void borrow(const te_problem &src) { p = src; }
  void take(const te_problem &src) {
    p = src;
    p.mem = TE_MEM_HOST;
    const size_t o = src.o, v = src.v, n = src.naux;
    auto cp = [&](int slot, const double *x, size_t cnt, const double **dst) {
      if (!x) { *dst = nullptr; return; }
      a[slot].assign(x, x + cnt);
      *dst = a[slot].data();
    };
    cp(0, src.eps_occ, o, &p.eps_occ);
    cp(1, src.eps_vir, v, &p.eps_vir);
    cp(2, src.t1, o * v, &p.t1);
    cp(3, src.t2, o * o * v * v, &p.t2);
    if (n > 0) {
      cp(4, src.B_oo, n * o * o, &p.B_oo);
      cp(5, src.B_ov, n * o * v, &p.B_ov);
      cp(6, src.B_vv, n * v * v, &p.B_vv);
      p.ovvv = p.ovoo = p.ovov = nullptr;
    } else {
      cp(7, src.ovvv, o * v * v * v, &p.ovvv);
      cp(8, src.ovoo, o * v * o * o, &p.ovoo);
      cp(9, src.ovov, o * v * o * v, &p.ovov);
      p.B_oo = p.B_ov = p.B_vv = nullptr;
    }
  }
  void drop() {
    for (auto &x : a) std::vector<double>().swap(x);
  }
};

enum class JS { Queued, Staging, Resident, Finishing, Done };

struct SJob {
  uint64_t ticket = 0;
  Prec prec = Prec::F64;
  HostCopy hc;
  int o = 0, v = 0, naux = 0;
  size_t footprint = 0;
  std::unique_ptr<Job> job;
  std::vector<int> trip;
  long ntr = 0, next = 0;
  DBuf eout, esum;
  double *h_E = nullptr;
  hipEvent_t done_ev = nullptr;
  JS state = JS::Queued;
  te_status status = TE_PENDING;
  std::string err;
  double E = 0.0;
  te_stats st{};
  clk::time_point t_submit, t_admit, t_staged, t_done;
  uint64_t retry_after = 0;  // requeued after a fragmented-arena miss
};

// Per-round limits. te_submit rejects jobs whose single triple would
// exceed them, so every round can hold at least one item.
constexpr int MAX_ITEMS = 4096;
constexpr int NSLOT = 3;   // rounds in flight
constexpr long MAX_TILES = 262144;
constexpr long MAX_BLKS = 2L << 20;

struct Slot {
  DBuf W, part, witems, eitems, ritems, tmap, bmap;
  WItem *h_wi = nullptr;
  EItem *h_ei = nullptr;
  RItem *h_ri = nullptr;
  int *h_tmap = nullptr, *h_bmap = nullptr;
  hipEvent_t ev_w = nullptr, ev_e = nullptr;
  bool busy = false;
};

}  // namespace

struct ServerImpl {
  int device = 0;
  size_t budget = 0, wcap = 0;
  int max_resident = 64, max_queued = 4096;
  bool borrow = false;
  int nstage = 2;
  Arena arena;
  // W builds on s_w, energy and reductions on s_e. (Two W streams, letting
  // a round's last partial wave of workgroups overlap the next round,
  // measured slower: concurrent W builds of different rounds share L2 and
  // slow the energy launches beside them more than the tails cost.)
  hipStream_t s_w[1] = {nullptr}, s_e = nullptr;
  std::vector<hipStream_t> s_stage;   // one staging stream per staging thread
  Slot slot[NSLOT];
  long round = 0;

  std::mutex mu;
  std::condition_variable cv;       // wakes the scheduler and the stager
  std::condition_variable cv_done;  // wakes te_wait callers
  bool stop = false;
  uint64_t next_ticket = 1;
  std::deque<SJob *> queue;         // submitted, not yet admitted
  std::list<SJob *> resident;       // staged (or staging), admission order
  std::unordered_map<uint64_t, std::unique_ptr<SJob>> jobs;
  size_t reserved = 0;              // footprints of admitted jobs
  uint64_t retired = 0;             // jobs retired so far
  std::thread sched;
  std::vector<std::thread> stagers;
  std::string fatal;

  void start();
  void shutdown();
  void stage_loop(int q);
  void sched_loop();
  enum class Launch { Done, NoWork, SlotBusy };
  Launch launch_round();
  void retire();
  void finish_job(SJob *j, te_status s, const std::string &msg);
  void fail_all(te_status s, const std::string &msg);
};

void ServerImpl::finish_job(SJob *j, te_status s, const std::string &msg) {
  j->status = s;
  j->err = msg;
  j->state = JS::Done;
  j->t_done = clk::now();
}

// Staging thread: admits jobs in arrival order while their footprint fits.
void ServerImpl::stage_loop(int q) {
  HIPCHK(hipSetDevice(device));
  hipStream_t ss = s_stage[q];
  for (;;) {
    SJob *j = nullptr;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv.wait(lk, [&] {
        if (stop) return true;
        if (queue.empty()) return false;
        if ((int)resident.size() >= max_resident) return false;
        if (queue.front()->retry_after > retired) return false;
        return reserved + queue.front()->footprint <= arena.cap;
      });
      if (stop) return;
      j = queue.front();
      queue.pop_front();
      j->state = JS::Staging;
      j->t_admit = clk::now();
      reserved += j->footprint;
      resident.push_back(j);
    }
    te_status s = TE_OK;
    std::string msg;
    try {
      JobOpts jo;
      jo.arena = &arena;
      jo.stream = ss;
      jo.budget = j->footprint;
      jo.drop_fp64_x = true;
      jo.prec = j->prec;
      te_config cfg{};
      cfg.device = device;
      cfg.x_mode = TE_X_RESIDENT;
      j->job.reset(make_job(&j->hc.p, &cfg, &jo));
      Job &J = *j->job;
      jalloc(J, j->eout, (size_t)j->ntr * 8);
      jalloc(J, j->esum, 8);
      HIPCHK(hipStreamSynchronize(ss));
      J.s_main = nullptr;  // the job's device work is tracked by server events from now on
      j->hc.drop();
    } catch (const Fail &f) {
      s = f.s;
      msg = f.msg;
    } catch (...) {
      s = TE_EDEVICE;
      msg = "staging failed";
    }
    std::lock_guard<std::mutex> lk(mu);
    j->t_staged = clk::now();
    if (!fatal.empty() && s == TE_OK) {   // the server failed while this job staged
      s = TE_EDEVICE;
      msg = fatal;
    }
    if (s == TE_ENOMEM && resident.size() > 1 && fatal.empty()) {
      // the arena is fragmented by other resident jobs: retry after one retires
      resident.remove(j);
      j->eout.release();
      j->esum.release();
      j->job.reset();
      reserved -= j->footprint;
      j->state = JS::Queued;
      j->retry_after = retired + 1;
      queue.push_front(j);
      cv.notify_all();
      continue;
    }
    if (s != TE_OK) {
      resident.remove(j);
      j->eout.release();
      j->esum.release();
      j->job.reset();
      reserved -= j->footprint;
      finish_job(j, s, msg);
      cv_done.notify_all();
    } else {
      j->state = JS::Resident;
    }
    cv.notify_all();
  }
}

// Build and launch one packed round into the next slot.
ServerImpl::Launch ServerImpl::launch_round() {
  Slot &S = slot[round % NSLOT];
  hipStream_t sw = s_w[0];
  if (S.busy) {
    if (hipEventQuery(S.ev_e) != hipSuccess) return Launch::SlotBusy;
    S.busy = false;
  }
  std::vector<SJob *> cand;
  Prec P = Prec::F64;
  {
    std::lock_guard<std::mutex> lk(mu);
    for (SJob *j : resident)
      if (j->state == JS::Resident && j->next < j->ntr) {
        if (cand.empty()) P = j->prec;
        if (j->prec == P) cand.push_back(j);
      }
  }
  if (cand.empty()) return Launch::NoWork;

  const int osz = out_bytes(P);
  // each job keeps the tile shape te_energy uses for its vp (the column-block
  // count that wastes least of its lone index); the round's W build is one
  // launch per shape
  struct Pick { SJob *j; long t; int nb; };
  std::vector<Pick> picks;
  long tiles = 0, blks = 0;
  size_t wbytes = 0;
  auto cfg_of = [&](SJob *j) { return wbuild_config(P, j->job->vp); };
  auto tiles_of = [&](SJob *j) {
    const long vp = j->job->vp;
    const WConfig c = cfg_of(j);
    return 3 * ((vp * vp + c.bm() - 1) / c.bm()) * ((vp + c.bn() - 1) / c.bn());
  };
  auto fits = [&](SJob *j) {
    const size_t vp = j->job->vp;
    if ((int)picks.size() >= MAX_ITEMS) return false;
    return tiles + tiles_of(j) <= MAX_TILES && blks + j->job->nsext <= MAX_BLKS &&
           wbytes + 3 * vp * vp * vp * osz <= wcap;
  };
  auto take = [&](SJob *j) {
    const size_t vp = j->job->vp;
    picks.push_back({j, j->next, cfg_of(j).nb});
    tiles += tiles_of(j);
    blks += j->job->nsext;
    wbytes += 3 * vp * vp * vp * osz;
    j->next++;
  };
  // Small jobs first (those whose remaining work fits a quarter of a round,
  // smallest first): they finish within a round or two. The rest of a round
  // goes to the large jobs in admission order, so a round mostly holds one
  // large job's triples in its i-major order (its X slices stay hot in L2
  // and the MALL across rounds, as in a job run alone) and no large job is
  // overtaken by a later one. (Every resident job in every round cost the
  // 16-bit W build and the energy kernel up to 2x their time alone; pure
  // shortest-remaining-work-first let later large jobs starve earlier ones
  // under Poisson arrivals.)
  std::vector<std::pair<long, SJob *>> small;
  std::vector<SJob *> large;
  for (SJob *j : cand) {   // cand is in admission order
    const long rem = (j->ntr - j->next) * tiles_of(j);
    if (rem <= MAX_TILES / 4) small.push_back({rem, j}); else large.push_back(j);
  }
  std::stable_sort(small.begin(), small.end(),
                   [](const auto &a, const auto &b) { return a.first < b.first; });
  for (auto &sj : small)
    while (sj.second->next < sj.second->ntr && fits(sj.second)) take(sj.second);
  for (SJob *j : large)
    while (j->next < j->ntr && fits(j)) take(j);
  if (picks.empty()) return Launch::NoWork;
  // items grouped by tile shape (order within a job's triples is kept; each
  // item's result is independent of its place in the round)
  std::stable_sort(picks.begin(), picks.end(),
                   [](const Pick &a, const Pick &b) { return a.nb < b.nb; });

  // items and maps in pinned memory
  const int n = (int)picks.size();
  long b0 = 0;
  size_t woff = 0;
  for (int q = 0; q < n; ++q) {
    SJob *j = picks[q].j;
    Job &J = *j->job;
    const Operands &op = J.op[(int)P];
    const long t = picks[q].t;
    const int i = j->trip[3 * t], jj = j->trip[3 * t + 1], k = j->trip[3 * t + 2];
    const size_t vp = J.vp, vp3 = vp * vp * vp;
    const size_t es = (P == Prec::F64) ? 8 : (P == Prec::F32 ? 4 : 2);
    void *W = S.W.as<char>() + woff;
    woff += 3 * vp3 * osz;
    WItem &w = S.h_wi[q];
    w.Xs[0] = (const char *)op.X + (size_t)i * vp3 * es;
    w.Xs[1] = (const char *)op.X + (size_t)jj * vp3 * es;
    w.Xs[2] = (const char *)op.X + (size_t)k * vp3 * es;
    w.In = op.In;
    w.xps = op.xps; w.ips = op.ips; w.lo = op.lo; w.scale = op.scale;
    w.W = W; w.o = J.o; w.vp = (int)vp; w.i = i; w.j = jj; w.k = k;
    resident_t2_views(J, op, P, w);
    WConfig wc = wbuild_config(P, (int)vp);
    w.mt = (int)((vp * vp + wc.bm() - 1) / wc.bm());
    w.nt = (int)((vp + wc.bn() - 1) / wc.bn());
    EItem &e = S.h_ei[q];
    e.W = W; resident_k_views(J, i, jj, k, e); e.t1 = J.t1.as<double>();
    e.eo = J.eo.as<double>(); e.ev = J.ev.as<double>(); e.sext = J.sext.as<int>();
    e.part = S.part.as<double>() + b0;
    e.part5 = S.part.as<double>() + MAX_BLKS + b0;
    e.o = J.o; e.v = J.v; e.vp = (int)vp; e.nT = (int)(vp / BOX);
    e.i = i; e.j = jj; e.k = k; e.nsext = J.nsext;
    for (long x = 0; x < J.nsext; ++x) S.h_bmap[b0 + x] = q;
    RItem &r = S.h_ri[q];
    r.part = e.part; r.part5 = e.part5; r.out = j->eout.as<double>() + t; r.n = J.nsext;
    r.out4 = r.out5 = nullptr;
    r.w = 2.0 - (i == jj) - (jj == k);
    b0 += J.nsext;
  }
  // tile maps, one region per shape group: [tiles of the group] item (local
  // to the group) of each tile, then [items of the group] first tile of each
  struct Group { int q0, nq, nb; long m0, ntl; };
  std::vector<Group> groups;
  long moff = 0;
  for (int q = 0; q < n;) {
    int qe = q;
    while (qe < n && picks[qe].nb == picks[q].nb) ++qe;
    Group G{q, qe - q, picks[q].nb, moff, 0};
    for (int x = q; x < qe; ++x) G.ntl += 3L * S.h_wi[x].mt * S.h_wi[x].nt;
    long tt = 0;
    for (int x = q; x < qe; ++x) {
      const long nt_ = 3L * S.h_wi[x].mt * S.h_wi[x].nt;
      for (long y = 0; y < nt_; ++y) S.h_tmap[moff + tt + y] = x - q;
      S.h_tmap[moff + G.ntl + (x - q)] = (int)tt;
      tt += nt_;
    }
    moff += G.ntl + G.nq;
    groups.push_back(G);
    q = qe;
  }
  for (int q = 0, acc = 0; q < n; ++q) {
    S.h_bmap[b0 + q] = acc;
    acc += S.h_ei[q].nsext;
  }
  HIPCHK(hipMemcpyAsync(S.witems.p, S.h_wi, n * sizeof(WItem), hipMemcpyHostToDevice, sw));
  HIPCHK(hipMemcpyAsync(S.tmap.p, S.h_tmap, moff * sizeof(int), hipMemcpyHostToDevice, sw));
  HIPCHK(hipMemcpyAsync(S.eitems.p, S.h_ei, n * sizeof(EItem), hipMemcpyHostToDevice, sw));
  HIPCHK(hipMemcpyAsync(S.ritems.p, S.h_ri, n * sizeof(RItem), hipMemcpyHostToDevice, sw));
  HIPCHK(hipMemcpyAsync(S.bmap.p, S.h_bmap, (b0 + n) * sizeof(int), hipMemcpyHostToDevice, sw));
  for (const Group &G : groups) {
    WConfig gc = wbuild_config(P, S.h_wi[G.q0].vp);
    gc.nb = G.nb;
    HIPCHK(launch_wbuild(P, S.witems.as<WItem>() + G.q0, S.tmap.as<int>() + G.m0, G.nq, 0,
                         G.ntl, gc, sw));
  }
  HIPCHK(hipEventRecord(S.ev_w, sw));
  HIPCHK(hipStreamWaitEvent(s_e, S.ev_w, 0));
  HIPCHK(launch_energy(P == Prec::F64, S.eitems.as<EItem>(), S.bmap.as<int>(), n, 0, b0, s_e));
  HIPCHK(launch_reduce(S.ritems.as<RItem>(), n, s_e));
  // jobs whose last triple is in this round: final fixed-order sum
  {
    std::lock_guard<std::mutex> lk(mu);
    for (SJob *j : cand) {
      if (j->next == j->ntr && j->state == JS::Resident) {
        HIPCHK(launch_sum(j->eout.as<double>(), j->ntr, j->esum.as<double>(), s_e));
        HIPCHK(hipMemcpyAsync(j->h_E, j->esum.p, 8, hipMemcpyDeviceToHost, s_e));
        HIPCHK(hipEventRecord(j->done_ev, s_e));
        j->state = JS::Finishing;
      }
    }
  }
  HIPCHK(hipEventRecord(S.ev_e, s_e));
  S.busy = true;
  round++;
  return Launch::Done;
}

void ServerImpl::retire() {
  std::vector<SJob *> fin;
  {
    std::lock_guard<std::mutex> lk(mu);
    for (SJob *j : resident)
      if (j->state == JS::Finishing && hipEventQuery(j->done_ev) == hipSuccess) fin.push_back(j);
  }
  for (SJob *j : fin) {
    const double E = *j->h_E;
    std::lock_guard<std::mutex> lk(mu);
    j->E = E;
    j->eout.release();
    j->esum.release();
    j->job.reset();
    reserved -= j->footprint;
    resident.remove(j);
    retired++;
    finish_job(j, TE_OK, "");
    const double lat = std::chrono::duration<double>(j->t_done - j->t_submit).count();
    const double svc = std::chrono::duration<double>(j->t_done - j->t_admit).count();
    j->st.seconds = lat;
    j->st.stage_seconds = std::chrono::duration<double>(j->t_staged - j->t_admit).count();
    j->st.n_triples = j->ntr;
    j->st.flops = (double)j->ntr * flops_per_triple(j->o, j->v);
    j->st.tflops = j->st.flops / std::max(svc, 1e-12) / 1e12;
  }
  if (!fin.empty()) {
    cv.notify_all();
    cv_done.notify_all();
  }
}

void ServerImpl::sched_loop() {
  try {
    HIPCHK(hipSetDevice(device));
    for (;;) {
      retire();
      const Launch l = launch_round();
      if (l == Launch::SlotBusy) {
        // every slot is queued on the device: block until the oldest drains,
        // then fill it at once (no polling gap between rounds)
        HIPCHK(hipEventSynchronize(slot[round % NSLOT].ev_e));
      }
      std::unique_lock<std::mutex> lk(mu);
      if (stop) break;
      if (l == Launch::NoWork) cv.wait_for(lk, std::chrono::microseconds(200));
    }
  } catch (const Fail &f) {
    fail_all(f.s, f.msg);
  }
}

// A device failure ends the server: no more staging or admission, the
// device work in flight drains before any job's memory is released, and
// every job ends with the error. A job a stager is still staging is left to
// that stager, which finishes it (stage_loop checks `fatal`) so that no
// caller can collect and free it under the stager's feet.
void ServerImpl::fail_all(te_status s, const std::string &msg) {
  {
    std::lock_guard<std::mutex> lk(mu);
    fatal = msg;
    stop = true;
    queue.clear();
  }
  cv.notify_all();
  (void)hipSetDevice(device);
  for (hipStream_t st : s_w)
    if (st) (void)hipStreamSynchronize(st);
  if (s_e) (void)hipStreamSynchronize(s_e);
  std::lock_guard<std::mutex> lk(mu);
  for (auto it = resident.begin(); it != resident.end();) {
    SJob *j = *it;
    if (j->state == JS::Staging) { ++it; continue; }
    j->eout.release();
    j->esum.release();
    j->job.reset();
    reserved -= j->footprint;
    it = resident.erase(it);
  }
  for (auto &kv : jobs) {
    SJob *j = kv.second.get();
    if (j->state != JS::Done && j->state != JS::Staging) finish_job(j, s, msg);
  }
  cv_done.notify_all();
}

void ServerImpl::start() {
  HIPCHK(hipSetDevice(device));
  for (hipStream_t &st : s_w) HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  HIPCHK(hipStreamCreateWithFlags(&s_e, hipStreamNonBlocking));
  s_stage.assign(nstage, nullptr);
  for (auto &st : s_stage) HIPCHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  // W scratch per round slot: large rounds keep the last, partly filled
  // wave of workgroups a small share of each W launch
  wcap = std::min<size_t>((size_t)8 << 30, budget / 12);
  for (Slot &S : slot) {
    S.W.alloc(wcap, nullptr, 0);
    S.part.alloc(2 * (size_t)MAX_BLKS * 8, nullptr, 0);
    S.witems.alloc(MAX_ITEMS * sizeof(WItem), nullptr, 0);
    S.eitems.alloc(MAX_ITEMS * sizeof(EItem), nullptr, 0);
    S.ritems.alloc(MAX_ITEMS * sizeof(RItem), nullptr, 0);
    S.tmap.alloc((MAX_TILES + MAX_ITEMS) * 4, nullptr, 0);
    S.bmap.alloc((MAX_BLKS + MAX_ITEMS) * 4, nullptr, 0);
    HIPCHK(hipHostMalloc((void **)&S.h_wi, MAX_ITEMS * sizeof(WItem), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void **)&S.h_ei, MAX_ITEMS * sizeof(EItem), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void **)&S.h_ri, MAX_ITEMS * sizeof(RItem), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void **)&S.h_tmap, S.tmap.bytes, hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void **)&S.h_bmap, S.bmap.bytes, hipHostMallocDefault));
    HIPCHK(hipEventCreateWithFlags(&S.ev_w, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&S.ev_e, hipEventDisableTiming));
  }
  const size_t scratch = NSLOT * (wcap + 2 * MAX_BLKS * 8 + (MAX_BLKS + MAX_ITEMS) * 4);
  if (budget <= scratch + ((size_t)1 << 28))
    throw Fail(TE_ENOMEM, "HBM budget too small for the server's round scratch");
  arena.init(budget - scratch);
  for (int q = 0; q < nstage; ++q) stagers.emplace_back([this, q] { stage_loop(q); });
  sched = std::thread([this] { sched_loop(); });
}

void ServerImpl::shutdown() {
  {
    std::lock_guard<std::mutex> lk(mu);
    stop = true;
  }
  cv.notify_all();
  for (auto &t : stagers)
    if (t.joinable()) t.join();
  if (sched.joinable()) sched.join();
  (void)hipSetDevice(device);
  for (hipStream_t st : s_w)
    if (st) (void)hipStreamSynchronize(st);
  if (s_e) (void)hipStreamSynchronize(s_e);
  for (auto st : s_stage)
    if (st) (void)hipStreamSynchronize(st);
  {
    std::lock_guard<std::mutex> lk(mu);
    for (auto &kv : jobs) {
      SJob *j = kv.second.get();
      j->eout.release();
      j->esum.release();
      j->job.reset();
      if (j->state != JS::Done) finish_job(j, TE_ECANCELED, "server destroyed");
      if (j->done_ev) (void)hipEventDestroy(j->done_ev);
      if (j->h_E) (void)hipHostFree(j->h_E);
      j->done_ev = nullptr;
      j->h_E = nullptr;
    }
  }
  cv_done.notify_all();
  for (Slot &S : slot) {
    S.W.release(); S.part.release(); S.witems.release(); S.eitems.release();
    S.ritems.release(); S.tmap.release(); S.bmap.release();
    if (S.h_wi) (void)hipHostFree(S.h_wi);
    if (S.h_ei) (void)hipHostFree(S.h_ei);
    if (S.h_ri) (void)hipHostFree(S.h_ri);
    if (S.h_tmap) (void)hipHostFree(S.h_tmap);
    if (S.h_bmap) (void)hipHostFree(S.h_bmap);
    if (S.ev_w) (void)hipEventDestroy(S.ev_w);
    if (S.ev_e) (void)hipEventDestroy(S.ev_e);
  }
  arena.destroy();
  for (hipStream_t st : s_w)
    if (st) (void)hipStreamDestroy(st);
  if (s_e) (void)hipStreamDestroy(s_e);
  for (auto st : s_stage)
    if (st) (void)hipStreamDestroy(st);
}

}  // namespace te

using namespace te;

extern "C" {

te_status te_server_create(const te_server_config *cfg_in, te_server *out) {
  TE_GUARD_BEGIN
  if (!out) return set_error(TE_EINVAL, "out is NULL");
  te_server_config cfg{};
  if (cfg_in) cfg = *cfg_in;
  if (cfg.max_resident_jobs < 0 || cfg.max_queued_jobs < 0)
    return set_error(TE_EINVAL, "negative limits");
  int ndev = 0;
  HIPCHK(hipGetDeviceCount(&ndev));
  if (cfg.device < 0 || cfg.device >= ndev) return set_error(TE_EINVAL, "bad device ordinal");
  HIPCHK(hipSetDevice(cfg.device));
  std::unique_ptr<ServerImpl> S(new ServerImpl());
  S->device = cfg.device;
  size_t freeb = 0, total = 0;
  HIPCHK(hipMemGetInfo(&freeb, &total));
  S->budget = cfg.hbm_budget ? cfg.hbm_budget : (size_t)(0.8 * (double)freeb);
  if (S->budget > freeb) return set_error(TE_ENOMEM, "HBM budget exceeds free device memory");
  S->max_resident = cfg.max_resident_jobs ? cfg.max_resident_jobs : 64;
  S->max_queued = cfg.max_queued_jobs ? cfg.max_queued_jobs : 4096;
  S->borrow = cfg.borrow_inputs != 0;
  if (cfg.staging_threads < 0 || cfg.staging_threads > 16)
    return set_error(TE_EINVAL, "staging_threads must be in [0, 16]");
  S->nstage = cfg.staging_threads ? cfg.staging_threads : 2;
  try {
    S->start();
  } catch (...) {
    S->shutdown();
    throw;
  }
  *out = reinterpret_cast<te_server>(S.release());
  return TE_OK;
  TE_GUARD_END
}

te_status te_submit(te_server srv, const te_problem *prob, te_precision prec, uint64_t *ticket) {
  TE_GUARD_BEGIN
  if (!srv || !ticket) return set_error(TE_EINVAL, "server and ticket are required");
  ServerImpl &S = *reinterpret_cast<ServerImpl *>(srv);
  if (!prob) return set_error(TE_EINVAL, "problem is NULL");
  if (prob->mem != TE_MEM_HOST) return set_error(TE_EINVAL, "te_submit takes host arrays");
  if (prec < TE_FP64 || prec > TE_FP16X2) return set_error(TE_EINVAL, "bad precision");
  if (prob->o < 1 || prob->v < 1 || prob->naux < 0)
    return set_error(TE_EINVAL, "need o >= 1, v >= 1, naux >= 0");
  if (!prob->eps_occ || !prob->eps_vir || !prob->t1 || !prob->t2)
    return set_error(TE_EINVAL, "eps_occ, eps_vir, t1 and t2 are required");
  if (prob->naux > 0 && (!prob->B_oo || !prob->B_ov || !prob->B_vv))
    return set_error(TE_EINVAL, "naux > 0 needs B_oo, B_ov and B_vv");
  if (prob->naux == 0 && (!prob->ovvv || !prob->ovoo || !prob->ovov))
    return set_error(TE_EINVAL, "naux == 0 needs ovvv, ovoo and ovov");
  if (pad_v(prob->v) / BOX > 1023) return set_error(TE_EINVAL, "v above 8184 is not supported");
  const Prec P = static_cast<Prec>(prec);
  const size_t fp = job_footprint(prob->o, prob->v, prob->naux, P);
  const size_t vp = pad_v(prob->v);
  if (fp > S.arena.cap || 3 * vp * vp * vp * (size_t)out_bytes(P) > S.wcap)
    return set_error(TE_ENOMEM, "job footprint " + std::to_string(fp) +
                                    " bytes can never fit the server budget");
  {
    const size_t bm = 128, nT = vp / BOX;   // smallest tile shape any precision uses
    const size_t tiles = 3 * ((vp * vp + bm - 1) / bm) * ((vp + 63) / 64);
    if (tiles > (size_t)MAX_TILES || nT * (nT + 1) * (nT + 2) / 6 > (size_t)MAX_BLKS)
      return set_error(TE_ENOMEM, "one triple of this job exceeds a server round");
  }
  {
    std::lock_guard<std::mutex> lk(S.mu);
    if (!S.fatal.empty()) return set_error(TE_EDEVICE, S.fatal);
    if (S.stop) return set_error(TE_EBUSY, "server is shutting down");
    if ((int)S.queue.size() >= S.max_queued) return set_error(TE_EBUSY, "queue is full");
  }
  std::unique_ptr<SJob> j(new SJob());
  j->t_submit = clk::now();
  j->prec = P;
  j->o = prob->o; j->v = prob->v; j->naux = prob->naux;
  j->footprint = fp;
  if (S.borrow)
    j->hc.borrow(*prob);
  else
    j->hc.take(*prob);
  j->trip = triple_list_host(prob->o);
  j->ntr = (long)j->trip.size() / 3;
  HIPCHK(hipSetDevice(S.device));
  HIPCHK(hipHostMalloc((void **)&j->h_E, 8, hipHostMallocDefault));
  HIPCHK(hipEventCreateWithFlags(&j->done_ev, hipEventDisableTiming));
  std::lock_guard<std::mutex> lk(S.mu);
  j->ticket = S.next_ticket++;
  *ticket = j->ticket;
  SJob *raw = j.get();
  S.jobs.emplace(j->ticket, std::move(j));
  if (raw->ntr == 0) {  // o = 1: only i=j=k, which contributes nothing
    raw->E = 0.0;
    S.finish_job(raw, TE_OK, "");
    S.cv_done.notify_all();
  } else {
    S.queue.push_back(raw);
    S.cv.notify_all();
  }
  return TE_OK;
  TE_GUARD_END
}

static te_status collect(ServerImpl &S, std::unique_lock<std::mutex> &lk, uint64_t ticket,
                         double *e_t, te_stats *st, bool block) {
  auto it = S.jobs.find(ticket);
  if (it == S.jobs.end()) return set_error(TE_ENOTFOUND, "unknown ticket");
  SJob *j = it->second.get();
  if (block) S.cv_done.wait(lk, [&] { return j->state == JS::Done; });
  if (j->state != JS::Done) return TE_PENDING;
  te_status s = j->status;
  if (s == TE_OK) {
    if (e_t) *e_t = j->E;
    if (st) *st = j->st;
  } else {
    set_error(s, j->err);
  }
  if (j->done_ev) (void)hipEventDestroy(j->done_ev);
  if (j->h_E) (void)hipHostFree(j->h_E);
  S.jobs.erase(it);
  return s;
}

te_status te_poll(te_server srv, uint64_t ticket, double *e_t, te_stats *st) {
  TE_GUARD_BEGIN
  if (!srv) return set_error(TE_EINVAL, "server is NULL");
  ServerImpl &S = *reinterpret_cast<ServerImpl *>(srv);
  std::unique_lock<std::mutex> lk(S.mu);
  return collect(S, lk, ticket, e_t, st, false);
  TE_GUARD_END
}

te_status te_wait(te_server srv, uint64_t ticket, double *e_t, te_stats *st) {
  TE_GUARD_BEGIN
  if (!srv) return set_error(TE_EINVAL, "server is NULL");
  ServerImpl &S = *reinterpret_cast<ServerImpl *>(srv);
  std::unique_lock<std::mutex> lk(S.mu);
  return collect(S, lk, ticket, e_t, st, true);
  TE_GUARD_END
}

te_status te_server_destroy(te_server srv) {
  TE_GUARD_BEGIN
  if (!srv) return set_error(TE_EINVAL, "server is NULL");
  ServerImpl *S = reinterpret_cast<ServerImpl *>(srv);
  S->shutdown();
  delete S;
  return TE_OK;
  TE_GUARD_END
}

}  // extern "C"
