"""CPU-side checks of the C ABI: the library loads, exports every function
include/te.h declares, and rejects bad arguments before touching a device."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2512_01055_amd import te

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "te.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(te_[a-z_]+)\s*\(", src)))


def test_header_declares_the_api():
    names = declared_functions()
    for required in ("te_init", "te_energy", "te_submit", "te_poll", "te_free"):
        assert required in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(te.LIB_PATH):
        pytest.skip("libte.so not built")
    out = subprocess.run(["nm", "-D", "--defined-only", te.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r"\bT (te_\w+)", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    lib = te.lib()
    for n in declared_functions():
        assert hasattr(lib, n)


def test_pure_functions():
    lib = te.lib()
    for o in (1, 2, 3, 6, 40, 100):
        n = lib.te_num_triples(o)
        assert n == o * (o + 1) * (o + 2) // 6 - o
    assert lib.te_num_triples(0) == 0
    t = te.triple_list(4)
    assert len(t) == lib.te_num_triples(4)
    assert all(i <= j <= k and not (i == j == k) for i, j, k in t)
    assert abs(lib.te_flops_per_triple(40, 400) - 12 * 400 ** 3 * 440) < 1
    assert lib.te_strerror(te.EINVAL) == b"invalid argument"


def test_argument_errors_need_no_device():
    lib = te.lib()
    h = C.c_void_p()
    assert lib.te_init(None, None, C.byref(h)) == te.EINVAL
    p = te.Problem()
    p.o, p.v, p.naux = 0, 10, 5
    assert lib.te_init(C.byref(p), None, C.byref(h)) == te.EINVAL
    assert b"o >= 1" in lib.te_last_error()
    x = np.zeros(100)
    p.o, p.v, p.naux = 2, 4, 3
    for n in ("eps_occ", "eps_vir", "t1", "t2", "B_oo", "B_ov"):
        setattr(p, n, x.ctypes.data)
    assert lib.te_init(C.byref(p), None, C.byref(h)) == te.EINVAL   # B_vv missing
    p.naux = 0
    assert lib.te_init(C.byref(p), None, C.byref(h)) == te.EINVAL   # explicit ints missing
    p.naux = -1
    assert lib.te_init(C.byref(p), None, C.byref(h)) == te.EINVAL
    p.naux, p.v = 3, 8185                 # vp / 8 box indices must fit 10 bits
    assert lib.te_init(C.byref(p), None, C.byref(h)) == te.EINVAL
    assert b"v above" in lib.te_last_error()
    p.v = 4
    # t2 in host memory: needs the factors, host arrays, and no resident slices
    p.naux = 3
    p.B_vv = x.ctypes.data
    for mem, naux, xmode in ((0, 0, 0), (1, 3, 0), (0, 3, 1)):
        p.mem, p.naux = mem, naux
        if naux == 0:
            for n in ("ovvv", "ovoo", "ovov"):
                setattr(p, n, x.ctypes.data)
        cfg = te.Config(0, None, 0, 0, xmode, 0, 1)
        assert lib.te_init(C.byref(p), C.byref(cfg), C.byref(h)) == te.EINVAL
        assert b"t2 in host memory" in lib.te_last_error()
    e = C.c_double()
    assert lib.te_energy(None, 0, C.byref(e), None, None) == te.EINVAL
    assert lib.te_free(None) == te.EINVAL
    assert lib.te_triple_list(0, None) == te.EINVAL


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(te, "_lib", None)
    monkeypatch.setattr(te, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="no fallback"):
        te.lib()


def test_slice_plan_counts():
    """On-the-fly schedule: a cache holding every slice assembles each once;
    smaller caches need more assemblies, never fewer than o."""
    lib = te.lib()
    for o in (3, 7, 20, 40):
        assert lib.te_plan_slice_loads(o, o, 1) == o
        assert lib.te_plan_slice_loads(o, o + 5, 64) == o
        prev = None
        for S in range(3, o + 1):
            n = lib.te_plan_slice_loads(o, S, 1)
            assert n >= o
            if prev is not None:
                assert n <= prev * 1.5 + 3        # no blow-up when the cache grows
            prev = n
    # blocked order keeps the o=100 schedule near o^3 / (6 (S/3)^2) block changes
    assert lib.te_plan_slice_loads(100, 45, 1) < 2000
    assert lib.te_plan_slice_loads(0, 10, 1) == -1
    assert lib.te_plan_slice_loads(10, 2, 1) == -1


# checkpoint files written from Python in the layout te.h documents
def _fnv(b: bytes, h: int = 1469598103934665603) -> int:
    for c in b:
        h = ((h ^ c) * 1099511628211) & (2 ** 64 - 1)
    return h


def _ckpt_header(o, v, naux, prec, tag, chunk):
    import struct
    n = o * (o + 1) * (o + 2) // 6 - o
    body = b"TECKPT01" + struct.pack("<iiiiQqq", o, v, naux, prec, tag, n, chunk)
    return body + struct.pack("<Q", _fnv(body)), n


def _ckpt_record(first, vals4, vals5):
    import struct
    body = struct.pack("<qq", first, len(vals4)) + struct.pack(f"<{len(vals4)}d", *vals4) \
        + struct.pack(f"<{len(vals5)}d", *vals5)
    return body + struct.pack("<Q", _fnv(body))


def test_checkpoint_scan_counts_intact_records(tmp_path):
    o, v, naux, chunk, tag = 4, 10, 7, 5, 99
    head, n = _ckpt_header(o, v, naux, 0, tag, chunk)
    assert n == 16                                   # 4 chunks: 5, 5, 5, 1
    recs = [_ckpt_record(f, [0.1 * f + q for q in range(min(chunk, n - f))],
                         [-q for q in range(min(chunk, n - f))]) for f in (0, 5, 10)]
    p = tmp_path / "run.ckpt"
    assert te.lib().te_checkpoint_scan(str(p).encode(), o, v, naux, 0, tag, chunk, None,
                                       None) == te.ENOTFOUND
    p.write_bytes(head + b"".join(recs))
    assert te.checkpoint_scan(str(p), o, v, naux, "fp64", chunk, tag) == (3, 4)
    # a torn last record does not count; the scan leaves the file as it is
    p.write_bytes(head + b"".join(recs)[:-3])
    assert te.checkpoint_scan(str(p), o, v, naux, "fp64", chunk, tag) == (2, 4)
    assert p.stat().st_size == len(head) + sum(map(len, recs)) - 3
    # a flipped byte ends the intact part at the record before it
    bad = bytearray(head + b"".join(recs))
    bad[len(head) + len(recs[0]) + 20] ^= 1
    p.write_bytes(bytes(bad))
    assert te.checkpoint_scan(str(p), o, v, naux, "fp64", chunk, tag) == (1, 4)
    # the last, shorter chunk and a duplicate record
    p.write_bytes(head + b"".join(recs) + _ckpt_record(15, [1.0], [2.0]) + recs[0])
    assert te.checkpoint_scan(str(p), o, v, naux, "fp64", chunk, tag) == (4, 4)


def test_checkpoint_scan_rejects_other_problems(tmp_path):
    o, v, naux, chunk = 4, 10, 7, 5
    head, _ = _ckpt_header(o, v, naux, 2, 5, chunk)
    p = tmp_path / "run.ckpt"
    p.write_bytes(head)
    assert te.checkpoint_scan(str(p), o, v, naux, "bf16x3", chunk, 5) == (0, 4)
    for args in ((o, v, naux, "fp64", chunk, 5), (o, v, naux, "bf16x3", chunk, 6),
                 (o, v + 1, naux, "bf16x3", chunk, 5), (o, v, naux, "bf16x3", chunk + 1, 5)):
        with pytest.raises(te.TeError) as ei:
            te.checkpoint_scan(str(p), *args)
        assert ei.value.status == te.EINVAL
    p.write_bytes(b"not a checkpoint at all" * 4)
    with pytest.raises(te.TeError) as ei:
        te.checkpoint_scan(str(p), o, v, naux, "bf16x3", chunk, 5)
    assert ei.value.status == te.EINVAL


def test_header_is_c99_and_library_links_from_c(tmp_path):
    """include/te.h is plain C; a C program links against libte.so and calls
    the entry points that need no device."""
    if not os.path.exists(te.LIB_PATH):
        pytest.skip("libte.so not built")
    src = tmp_path / "use_te.c"
    src.write_text(r'''
#include <stdio.h>
#include "te.h"
int main(void) {
  int32_t ijk[3 * 16];
  te_stats st;
  te_config cfg = {0};
  (void)st; (void)cfg;
  if (te_num_triples(4) != 16) return 1;
  if (te_triple_list(4, ijk) != TE_OK || ijk[0] != 0 || ijk[2] != 1) return 2;
  if (te_flops_per_triple(40, 400) != 12.0 * 400 * 400 * 400 * 440) return 3;
  if (te_init(NULL, NULL, NULL) != TE_EINVAL) return 4;
  printf("%s\n", te_strerror(TE_EIO));
  return 0;
}
''')
    exe = tmp_path / "use_te"
    libdir = os.path.dirname(te.LIB_PATH)
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-pedantic", str(src),
                        f"-I{os.path.join(ROOT, 'include')}", f"-L{libdir}", "-lte",
                        f"-Wl,-rpath,{libdir}", "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stderr)
    assert "checkpoint" in r.stdout


def test_checkpoint_scan_survives_corruption(tmp_path):
    """Random byte flips, truncations and appended garbage never crash the
    reader: it answers OK or EINVAL, and never counts more chunks than the
    intact records of the file hold."""
    o, v, naux, chunk, tag = 5, 12, 9, 4, 3
    head, n = _ckpt_header(o, v, naux, 0, tag, chunk)
    total = (n + chunk - 1) // chunk
    recs = [_ckpt_record(f, [1.0 + f + q for q in range(min(chunk, n - f))],
                         [2.0 - q for q in range(min(chunk, n - f))]) for f in range(0, n, chunk)]
    good = head + b"".join(recs)
    p = tmp_path / "fuzz.ckpt"
    rng = np.random.default_rng(11)
    for trial in range(300):
        b = bytearray(good)
        kind = trial % 3
        if kind == 0:
            for _ in range(int(rng.integers(1, 4))):
                b[int(rng.integers(len(b)))] ^= int(rng.integers(1, 256))
        elif kind == 1:
            b = b[:int(rng.integers(len(b) + 1))]
        else:
            b += rng.integers(0, 256, int(rng.integers(1, 200)), dtype=np.uint8).tobytes()
        p.write_bytes(bytes(b))
        done, tot = C.c_int64(-1), C.c_int64(-1)
        s = te.lib().te_checkpoint_scan(str(p).encode(), o, v, naux, 0, tag, chunk,
                                        C.byref(done), C.byref(tot))
        assert s in (te.OK, te.EINVAL), (trial, s)
        if s == te.OK:
            assert tot.value == total and 0 <= done.value <= total
            # records are checksummed: a scan never counts a record whose bytes changed
            intact = 0
            off = len(head)
            for r in recs:
                if bytes(b[off:off + len(r)]) != r:
                    break
                intact += 1
                off += len(r)
            assert done.value == intact, (trial, done.value, intact)
