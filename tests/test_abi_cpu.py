"""CPU checks of the C ABI library: it loads, exports every declared symbol,
and its host-only entry points (moduli, Richardson fit) agree with the
oracle.  No GPU compute is called."""
import ctypes as ct
import os
import re
import subprocess

import numpy as np
import pytest

from oracle import bounds, hier

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2208_02320_amd", "libhh.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libhh.so not built")


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "hh.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char \*|long long)\s*\*?\s*(hh_\w+)\(", txt, re.M)))


def test_header_declares_the_binding_symbols():
    from paper_2208_02320_amd import hh
    assert declared_symbols() == sorted(hh.SYMBOLS)


def test_library_exports_every_declared_symbol():
    lib = ct.CDLL(LIB)
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_binding_loads():
    from paper_2208_02320_amd import hh
    lib = hh.load_library()
    o = hh.default_opts()
    assert o.tol == 1e-6 and o.max_iter == 0 and o.stall_limit == 0 and o.scheme == 0 and o.precision == 0
    assert o.retry == 1 and o.verify == 0
    assert lib.hh_size_supported(256, 0) == 1 and lib.hh_size_supported(7, 0) == 0
    assert lib.hh_size_supported(80, 1) == 1 and lib.hh_size_supported(80, 2) == 0


def test_supported_sizes_are_the_documented_ones():
    """hh_size_supported answers exactly the lists of the header."""
    from paper_2208_02320_amd import hh
    lib = hh.load_library()
    text = open(os.path.join(ROOT, "include", "hh.h")).read()
    doc = text[text.index("1 if axis length n has compiled FFT passes"):text.index("int hh_size_supported")]
    f32 = [int(x) for x in re.search(r"FP32 \(precision 0\):([\d\s*]+)", doc).group(1).replace("*", " ").split()]
    f64 = [int(x) for x in re.search(r"FP64 \(precision 1\):([\d\s*]+)", doc).group(1).replace("*", " ").split()]
    assert [n for n in range(1, 1100) if lib.hh_size_supported(n, 0)] == f32
    assert [n for n in range(1, 1100) if lib.hh_size_supported(n, 1)] == f64


def test_moduli_host_entry_point():
    from paper_2208_02320_amd import hh
    C = bounds.iso_voigt_matrix(37.0, 44.0)
    K, G = hh.moduli(C)
    assert np.isclose(K, 37.0) and np.isclose(G, 44.0)
    rng = np.random.default_rng(0)
    A = rng.standard_normal((6, 6))
    C = A @ A.T + 6 * np.eye(6)
    assert np.allclose(hh.moduli(C), hier.voigt_moduli(C), rtol=1e-14)


def test_richardson_host_entry_point():
    from paper_2208_02320_amd import hh
    rng = np.random.default_rng(1)
    ns = [32, 64, 128]
    Cs = rng.standard_normal((3, 6, 6)) + 10
    Ci, sl = hh.richardson(ns, Cs)
    m, c = hier.richardson(ns, Cs.reshape(3, 36))
    assert np.allclose(Ci.ravel(), m, rtol=1e-12) and np.allclose(sl.ravel(), c, rtol=1e-10)
    with pytest.raises(hh.HHError):
        hh.richardson([32, 32], Cs[:2])


def test_mean_moduli_host_entry_point():
    """The AM comparator of Sec. 5 equals the oracle's arithmetic mean of the
    subimage moduli."""
    from paper_2208_02320_amd import hh
    rng = np.random.default_rng(2)
    A = rng.standard_normal((27, 6, 6))
    C = np.einsum("nij,nkj->nik", A, A) + 6 * np.eye(6)
    K, G = hh.mean_moduli(np.stack([hier.to21(c) for c in C]))
    assert np.allclose([K, G], hier.arithmetic_mean_moduli(C), rtol=1e-14)
    with pytest.raises(hh.HHError):
        hh.mean_moduli(np.zeros((0, 21)))


def test_context_needs_gpu():
    import torch
    from paper_2208_02320_amd import hh
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(RuntimeError):
        hh.Context(0)


def run_client(*args):
    exe = os.path.join(ROOT, "paper_2208_02320_amd", "examples", "hh_client")
    if not os.path.exists(exe):
        pytest.skip("C client not built")
    p = subprocess.run([exe] + [str(a) for a in args], capture_output=True, text=True, timeout=120)
    out = {}
    for line in p.stdout.splitlines():
        key, *vals = line.split()
        out[key] = [float(v) for v in vals]
    return p.returncode, out, p.stderr


def test_plain_c_client_host_entry_points():
    """A C program linked against libhh.so, without Python: the Voigt moduli
    of an isotropic matrix (lambda 2, mu 3) are K = lambda + 2 mu / 3 and
    G = mu; the n^-1 fit recovers M(n) = 5 + 40 / n exactly; a context needs
    a gfx950 device (HH_EDEVICE where there is none)."""
    rc, out, err = run_client("host")
    assert rc == 0, err
    assert out["supported_f32"] == [256, 1, 7, 0]
    assert np.allclose(out["moduli"], [4.0, 3.0], rtol=0, atol=1e-14)
    assert np.allclose(out["richardson"], [5.0, 40.0], rtol=1e-12)
    assert out["create"][0] in (0, -4)
    if out["create"][0] == -4:
        assert "hh_create:" in err  # the reason, read with hh_last_error(NULL)
