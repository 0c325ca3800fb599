"""The Python binding refuses host arrays of the wrong size before the
library reads them (the C interface takes plain pointers and reads exactly
N, 3 N or Q N elements).  Runs on the CPU: the checks come before any
library call, on a wrapper object that holds no handle."""
import numpy as np
import pytest

import paper_2112_08926_amd as lbm
from paper_2112_08926_amd import _lib


@pytest.fixture
def lat():
    g = object.__new__(lbm.Lattices)
    g.params = [lbm.make_params(8, 4, 2, q=19, storage="fp16s"), lbm.make_params(3, 3, 3, q=19, storage="fp16s")]
    g.q, g.storage, g.h = 19, g.params[0].storage, None
    return g


def test_wrong_sizes_refused(lat):
    n = 8 * 4 * 2
    with pytest.raises(ValueError, match="flags"):
        lat.set_boundaries(0, np.zeros(n - 1, np.uint8))
    with pytest.raises(ValueError, match="flags"):
        lat.set_boundaries(1, np.zeros(n, np.uint8))            # lattice 0's size for lattice 1
    with pytest.raises(ValueError, match="rho"):
        lat.set_rho_u(0, rho=np.ones(n + 1))
    with pytest.raises(ValueError, match="u"):
        lat.set_rho_u(0, u=np.zeros((2, n)))
    with pytest.raises(ValueError, match="u_ref"):
        lat.diagnostics(0, u_ref=np.zeros(n))
    with pytest.raises(ValueError, match="codes"):
        lat.set_ddf(0, np.zeros((18, n), np.uint16))


def test_sized_accepts_any_shape_of_the_right_size():
    a = np.arange(24, dtype=np.int64).reshape(2, 3, 4)
    c = _lib._sized(a, np.float64, 24, "x")
    assert c.dtype == np.float64 and c.flags.c_contiguous and np.array_equal(c, a.reshape(-1).astype(np.float64).reshape(2, 3, 4))
    f = np.asfortranarray(np.arange(6.0).reshape(2, 3))
    assert np.array_equal(_lib._sized(f, np.float64, 6, "x"), np.arange(6.0).reshape(2, 3))
