"""The plain C client of the ABI (paper_2208_02320_amd/examples/hh_client.c)
on the GPU: a process with no Python in it homogenizes a laminate through
host buffers, checked against the closed form the oracle pins."""
import numpy as np
import pytest

from oracle import bounds
from oracle import galerkin as g

from test_abi_cpu import run_client

pytestmark = pytest.mark.gpu


def test_plain_c_client_solves_a_laminate():
    """16^3 two-phase laminate (quartz 37/44, pore 2.25/1 GPa), 4-voxel layers
    normal to z: with even layer thickness the discrete solution is the
    layered closed form, and the two-level scheme with 8^3 blocks (each a
    whole period) gives it again."""
    rc, out, err = run_client("solve", 16, 4)
    assert rc == 0, err
    want = bounds.backus([0.5, 0.5], [(37.0, 44.0), (2.25, 1.0)])
    C = np.array(out["C"]).reshape(6, 6)
    C2 = np.array(out["C_two_level"]).reshape(6, 6)
    print("C client: laminate error %.2e, two-level %.2e, iters %s" %
          (g.rel_error(C, want), g.rel_error(C2, want), out["iters"]))
    assert g.rel_error(C, want) < 1e-5
    assert g.rel_error(C2, want) < 1e-5
