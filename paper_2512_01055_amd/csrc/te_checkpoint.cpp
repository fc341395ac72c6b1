// Checkpointed evaluation of a whole job: the triple list is cut into chunks
// of consecutive triples, and each finished chunk's per-triple E[4] / E[5]
// parts are appended to a file, so that a long run (hours at o = 100,
// v = 800) can stop - a crash, a wall-time limit - and resume without
// recomputing finished chunks.
//
// File layout (native byte order):
//   header  magic "TECKPT01", int32 o, v, naux, precision, uint64 tag,
//           int64 number of triples, int64 chunk, uint64 FNV-1a of the above
//   record  int64 first triple, int64 count, double e4[count],
//           double e5[count], uint64 FNV-1a of the record's other bytes
// A record is written whole and flushed to disk before the next chunk
// starts; a torn last record fails its checksum and is recomputed. A writer
// holds an exclusive advisory lock on the file, so that a second run on the
// same checkpoint is turned away instead of interleaving its records.
#include <fcntl.h>
#include <sys/file.h>
#include <sys/stat.h>
#include <unistd.h>

#include <cerrno>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <vector>

#include "te_job.h"

namespace te {
namespace {

constexpr char kMagic[8] = {'T', 'E', 'C', 'K', 'P', 'T', '0', '1'};

struct Header {
  char magic[8];
  int32_t o, v, naux, prec;
  uint64_t tag;
  int64_t ntriples, chunk;
  uint64_t check;
};
static_assert(sizeof(Header) == 56, "checkpoint header layout");

uint64_t fnv1a(const void *p, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char *c = static_cast<const unsigned char *>(p);
  for (size_t i = 0; i < n; ++i) {
    h ^= c[i];
    h *= 1099511628211ull;
  }
  return h;
}

Header make_header(int o, int v, int naux, int prec, uint64_t tag, int64_t n, int64_t chunk) {
  Header h;
  std::memset(&h, 0, sizeof h);
  std::memcpy(h.magic, kMagic, 8);
  h.o = o; h.v = v; h.naux = naux; h.prec = prec;
  h.tag = tag; h.ntriples = n; h.chunk = chunk;
  h.check = fnv1a(&h, offsetof(Header, check));
  return h;
}

struct Fd {
  int fd = -1;
  ~Fd() {
    if (fd >= 0) ::close(fd);
  }
};

[[noreturn]] void io_fail(const std::string &what, const char *path) {
  throw Fail(TE_EIO, what + " " + path + ": " + std::strerror(errno));
}

// Reads exactly n bytes; false on a short read (end of file).
bool read_all(int fd, void *p, size_t n, const char *path) {
  char *c = static_cast<char *>(p);
  while (n) {
    ssize_t r = ::read(fd, c, n);
    if (r < 0 && errno == EINTR) continue;
    if (r < 0) io_fail("read", path);
    if (r == 0) return false;
    c += r;
    n -= (size_t)r;
  }
  return true;
}

void write_all(int fd, const void *p, size_t n, const char *path) {
  const char *c = static_cast<const char *>(p);
  while (n) {
    ssize_t r = ::write(fd, c, n);
    if (r < 0 && errno == EINTR) continue;
    if (r < 0) io_fail("write", path);
    c += r;
    n -= (size_t)r;
  }
}

// Intact records of an open checkpoint positioned after its header: fills
// done / e4 / e5 and returns the offset where the intact part ends.
off_t scan_records(int fd, const Header &h, std::vector<char> &done, std::vector<double> &e4,
                   std::vector<double> &e5, const char *path) {
  const int64_t n = h.ntriples, chunk = h.chunk;
  off_t end = (off_t)sizeof(Header);
  std::vector<double> buf;
  for (;;) {
    int64_t fc[2];
    if (!read_all(fd, fc, sizeof fc, path)) break;
    const int64_t first = fc[0], count = fc[1];
    if (first < 0 || first >= n || first % chunk != 0 || count != std::min(chunk, n - first))
      break;
    buf.resize(2 * (size_t)count);
    uint64_t check = 0;
    if (!read_all(fd, buf.data(), buf.size() * 8, path)) break;
    if (!read_all(fd, &check, 8, path)) break;
    uint64_t c = fnv1a(fc, sizeof fc);
    c = fnv1a(buf.data(), buf.size() * 8, c);
    if (c != check) break;
    const int64_t ci = first / chunk;
    if (!done[ci]) {
      std::memcpy(&e4[first], buf.data(), (size_t)count * 8);
      std::memcpy(&e5[first], buf.data() + count, (size_t)count * 8);
      done[ci] = 1;
    }
    end += (off_t)(sizeof fc + buf.size() * 8 + 8);
  }
  return end;
}

// Reads and checks the header of an existing checkpoint against `want`.
void check_header(int fd, const Header &want, const char *path) {
  Header h;
  if (!read_all(fd, &h, sizeof h, path) || std::memcmp(h.magic, kMagic, 8) != 0 ||
      h.check != fnv1a(&h, offsetof(Header, check)))
    throw Fail(TE_EINVAL, std::string("not a (T) checkpoint file: ") + path);
  if (h.o != want.o || h.v != want.v || h.naux != want.naux || h.prec != want.prec ||
      h.tag != want.tag || h.ntriples != want.ntriples || h.chunk != want.chunk)
    throw Fail(TE_EINVAL, std::string("checkpoint ") + path +
                              " belongs to another problem, precision, tag or chunk size");
}

// Compensated (Neumaier) sum in index order.
double ordered_sum(const std::vector<double> &x) {
  double s = 0.0, c = 0.0;
  for (double a : x) {
    double t = s + a;
    c += std::abs(s) >= std::abs(a) ? (s - t) + a : (a - t) + s;
    s = t;
  }
  return s + c;
}

void add_stats(te_stats &a, const te_stats &b) {
  a.seconds += b.seconds;
  a.flops += b.flops;
  a.n_triples += b.n_triples;
  a.stage_seconds += b.stage_seconds;
  a.assemble_flops += b.assemble_flops;
  a.w_kernel_seconds += b.w_kernel_seconds;
  a.w_launches += b.w_launches;
  a.e_kernel_seconds += b.e_kernel_seconds;
  a.e_launches += b.e_launches;
  a.slices_assembled += b.slices_assembled;
  a.assemble_seconds += b.assemble_seconds;
  a.cache_slices = b.cache_slices;
  a.tflops = a.seconds > 0 ? a.flops / a.seconds / 1e12 : 0.0;
}

}  // namespace
}  // namespace te

using namespace te;

extern "C" {

te_status te_energy_checkpointed(te_job job, te_precision prec, const char *path, uint64_t tag,
                                 int64_t chunk, int64_t max_chunks, double *e_t, double *e4_sum,
                                 double *e5_sum, te_stats *st) {
  TE_GUARD_BEGIN
  if (!job || !path) return set_error(TE_EINVAL, "job and path are required");
  if (chunk < 1 || max_chunks < 0) return set_error(TE_EINVAL, "need chunk >= 1, max_chunks >= 0");
  Job &J = *reinterpret_cast<Job *>(job);
  const Prec p = to_prec(prec);
  const std::vector<int> t = triple_list_host(J.o);
  const int64_t n = (int64_t)t.size() / 3;
  const int64_t nchunks = (n + chunk - 1) / chunk;
  const Header want = make_header(J.o, J.v, J.naux, (int)prec, tag, n, chunk);

  Fd f;
  f.fd = ::open(path, O_RDWR | O_CREAT | O_CLOEXEC, 0644);
  if (f.fd < 0) io_fail("open", path);
  while (::flock(f.fd, LOCK_EX | LOCK_NB) != 0) {
    if (errno == EINTR) continue;
    if (errno == EWOULDBLOCK)
      return set_error(TE_EBUSY, std::string("checkpoint ") + path + " is in use by another run");
    io_fail("lock", path);
  }
  struct stat sb;
  if (::fstat(f.fd, &sb) != 0) io_fail("stat", path);
  std::vector<char> done((size_t)nchunks, 0);
  std::vector<double> e4((size_t)n, 0.0), e5((size_t)n, 0.0);
  if (sb.st_size < (off_t)sizeof(Header)) {
    // new file, or one torn while its header was written
    if (sb.st_size > 0) {
      char probe[8] = {0};
      if (!read_all(f.fd, probe, std::min<size_t>(8, (size_t)sb.st_size), path) ||
          std::memcmp(probe, kMagic, std::min<size_t>(8, (size_t)sb.st_size)) != 0)
        throw Fail(TE_EINVAL, std::string("not a (T) checkpoint file: ") + path);
    }
    if (::ftruncate(f.fd, 0) != 0) io_fail("truncate", path);
    if (::lseek(f.fd, 0, SEEK_SET) < 0) io_fail("seek", path);
    write_all(f.fd, &want, sizeof want, path);
    if (::fsync(f.fd) != 0) io_fail("fsync", path);
  } else {
    check_header(f.fd, want, path);
    const off_t end = scan_records(f.fd, want, done, e4, e5, path);
    if (end < sb.st_size && ::ftruncate(f.fd, end) != 0) io_fail("truncate", path);
    if (::lseek(f.fd, end, SEEK_SET) < 0) io_fail("seek", path);
  }

  HIPCHK(hipSetDevice(J.device));
  te_stats total{};
  int64_t fresh = 0;
  std::vector<double> rec;
  for (int64_t c = 0; c < nchunks; ++c) {
    if (done[c]) continue;
    if (max_chunks > 0 && fresh == max_chunks) break;
    const int64_t first = c * chunk, cnt = std::min(chunk, n - first);
    SplitOut so;
    so.pt4 = &e4[first];
    so.pt5 = &e5[first];
    te_stats s{};
    run_triples(J, p, t.data() + 3 * first, (long)cnt, nullptr, nullptr, &s, &so);
    add_stats(total, s);
    int64_t fc[2] = {first, cnt};
    rec.assign(e4.begin() + first, e4.begin() + first + cnt);
    rec.insert(rec.end(), e5.begin() + first, e5.begin() + first + cnt);
    uint64_t check = fnv1a(fc, sizeof fc);
    check = fnv1a(rec.data(), rec.size() * 8, check);
    std::vector<char> bytes(sizeof fc + rec.size() * 8 + 8);
    std::memcpy(bytes.data(), fc, sizeof fc);
    std::memcpy(bytes.data() + sizeof fc, rec.data(), rec.size() * 8);
    std::memcpy(bytes.data() + sizeof fc + rec.size() * 8, &check, 8);
    write_all(f.fd, bytes.data(), bytes.size(), path);
    if (::fsync(f.fd) != 0) io_fail("fsync", path);
    done[c] = 1;
    ++fresh;
  }
  if (st) *st = total;
  for (int64_t c = 0; c < nchunks; ++c)
    if (!done[c]) return TE_PENDING;
  const double E4 = ordered_sum(e4), E5 = ordered_sum(e5);
  if (e4_sum) *e4_sum = E4;
  if (e5_sum) *e5_sum = E5;
  if (e_t) *e_t = E4 + E5;
  return TE_OK;
  TE_GUARD_END
}

te_status te_checkpoint_scan(const char *path, int32_t o, int32_t v, int32_t naux,
                             te_precision prec, uint64_t tag, int64_t chunk, int64_t *chunks_done,
                             int64_t *chunks_total) {
  TE_GUARD_BEGIN
  if (!path || o < 1 || v < 1 || naux < 0 || chunk < 1)
    return set_error(TE_EINVAL, "need a path, o >= 1, v >= 1, naux >= 0, chunk >= 1");
  (void)to_prec(prec);
  const int64_t n = (int64_t)o * (o + 1) * (o + 2) / 6 - o;
  const int64_t nchunks = (n + chunk - 1) / chunk;
  const Header want = make_header(o, v, naux, (int)prec, tag, n, chunk);
  Fd f;
  f.fd = ::open(path, O_RDONLY | O_CLOEXEC);
  if (f.fd < 0) {
    if (errno == ENOENT) return set_error(TE_ENOTFOUND, std::string("no checkpoint at ") + path);
    io_fail("open", path);
  }
  check_header(f.fd, want, path);
  std::vector<char> done((size_t)nchunks, 0);
  std::vector<double> e4((size_t)n, 0.0), e5((size_t)n, 0.0);
  scan_records(f.fd, want, done, e4, e5, path);
  int64_t k = 0;
  for (char d : done) k += d;
  if (chunks_done) *chunks_done = k;
  if (chunks_total) *chunks_total = nchunks;
  return TE_OK;
  TE_GUARD_END
}

}  // extern "C"
