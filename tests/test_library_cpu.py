"""CPU-side checks of libhomotopy: it loads, exports every entry point the
header declares, and its host-only logic (path counts, batch layout,
duplicate detection, argument checks) behaves.  No GPU calls."""
import os
import re

import numpy as np
import pytest

import oracle
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def hp():
    import paper_1804_03807_amd as hp
    hp.load()
    return hp


def declared_functions():
    text = open(os.path.join(ROOT, "include", "homotopy.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hp_[a-z_0-9]+)\s*\(", text)))


def test_exports_every_declared_symbol(hp):
    import ctypes
    lib = ctypes.CDLL(hp._lib.SO_PATH)
    names = declared_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(hp._lib.EXPORTED) == names


def test_path_counts(hp):
    assert hp.path_count(W.cyclic8().systems[0]) == 40320
    assert hp.path_count(W.cyclic10().systems[0]) == 3628800
    assert hp.path_count(W.dense_small().systems[0]) == 32
    b = W.dense_batch(8)
    for s in b.systems:
        assert hp.path_count(s) == s.bezout()


def test_rejects_bad_systems(hp):
    s = W.cyclic_system(12, np.random.default_rng(0))
    assert hp.path_count(s) == 479001600
    bad = W.PolySystem(13, np.zeros(14, np.int32), np.zeros(0, np.complex128),
                       np.zeros((0, 13), np.uint8))
    assert hp.path_count(bad) == -1
    s2 = W.dense_system(3, [2, 2, 2], np.random.default_rng(1))
    s2.exps[0, 0] = 16  # exponent above the supported maximum
    assert hp.path_count(s2) == -1
    s3 = W.dense_system(3, [2, 2, 2], np.random.default_rng(1))
    s3.eq_ptr[1] = s3.eq_ptr[2] + 1  # not monotone
    assert hp.path_count(s3) == -1


def test_batch_layout(hp):
    b = W.dense_batch(5)
    po, xo = hp.batch_layout(b.systems)
    counts = [s.bezout() for s in b.systems]
    assert list(np.diff(po)) == counts
    assert list(np.diff(xo)) == [c * s.n for c, s in zip(counts, b.systems)]


def test_find_duplicates_matches_oracle(hp, oracle_lib):
    rng = np.random.default_rng(5)
    n, P = 4, 600
    x = (rng.standard_normal((P, n)) + 1j * rng.standard_normal((P, n))) * 3
    st = np.zeros(P, np.int32)
    st[::9] = 2  # not converged: ignored
    planted = set()
    for k in range(0, P // 2, 17):  # near-copies inside and outside 1e-6, no chains
        j = k + P // 2
        x[j] = x[k] * (1 + (3e-7 if k % 2 else 5e-6))
        if k % 2 and st[j] == 0 and st[k] == 0:
            planted.add((min(j, k), max(j, k)))
    got = {tuple(int(v) for v in p) for p in hp.find_duplicates(x, st)}
    ref = {tuple(int(v) for v in p) for p in oracle.find_duplicates(x, st)}
    assert got == ref == planted and len(planted) >= 5


@pytest.mark.parametrize("n", [3, 5, 8])
def test_specialised_kernel_compiles(hp, n):
    """The kernel specialised to a system's support is written and compiled
    for gfx950 by the library itself (hiprtc), without a device."""
    s = W.cyclic_system(n, np.random.default_rng(n))
    assert hp.spec_compile(s) > 1000
    d = W.dense_system(3, [3, 2, 2], np.random.default_rng(5))  # exponents above 1
    assert hp.spec_compile(d) > 1000


def test_specialised_kernel_forms_compile(hp):
    """The plans', the server's and the coefficient-parameter forms compile
    (hiprtc, no device); another form number is an argument error."""
    s = W.cyclic_system(5, np.random.default_rng(9))
    sizes = [hp.spec_compile(s, form=f) for f in (0, 1, 2)]
    assert all(b > 1000 for b in sizes)
    assert sizes[0] == hp.spec_compile(s)
    with pytest.raises(hp.HomotopyError) as e:
        hp.spec_compile(s, form=3)
    assert e.value.code == hp._lib.HP_E_INVALID_ARG


def test_specialised_kernel_limits(hp):
    """n above 10 and systems with more than 1024 factors in all have none."""
    with pytest.raises(hp.HomotopyError) as e:
        hp.spec_compile(W.cyclic_system(11, np.random.default_rng(0)))
    assert e.value.code == hp._lib.HP_E_UNSUPPORTED_N
    big = W.dense_system(8, [3] * 8, np.random.default_rng(0))  # 8 x 165 terms
    with pytest.raises(hp.HomotopyError) as e:
        hp.spec_compile(big)
    assert e.value.code == hp._lib.HP_E_UNSUPPORTED_N


def test_specialised_kernel_disk_cache(hp, tmp_path):
    """With $HP_JIT_CACHE set, the compiled code objects (the plans' and the
    server's form) are written there and a fresh process loads them instead
    of compiling (same code size)."""
    import subprocess
    import sys
    s = W.dense_system(2, [2, 3], np.random.default_rng(77))  # a support no other test uses
    env = dict(os.environ, HP_JIT_CACHE=str(tmp_path))
    code = ("import sys, time; sys.path.insert(0, %r); import numpy as np; import workloads as W; "
            "import paper_1804_03807_amd as hp; "
            "s = W.dense_system(2, [2, 3], np.random.default_rng(77)); "
            "t = time.perf_counter(); b = hp.spec_compile(s); "
            "print(b, time.perf_counter() - t)" % ROOT)
    out1 = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                          timeout=300, check=True).stdout.split()
    files = sorted(tmp_path.glob("hp_spec_*.bin"))
    assert len(files) == 2 and max(f.stat().st_size for f in files) > int(out1[0])
    ino = [f.stat().st_ino for f in files]
    out2 = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                          timeout=300, check=True).stdout.split()
    assert out2[0] == out1[0]
    # loaded, not compiled: a compilation would have replaced the files
    assert sorted(tmp_path.glob("hp_spec_*.bin")) == files
    assert [f.stat().st_ino for f in files] == ino
    assert hp.spec_compile(s) == int(out1[0])
