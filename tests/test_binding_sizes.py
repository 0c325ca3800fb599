"""The Python binding refuses host arrays of the wrong size before the
library reads them (the C interface takes plain pointers and reads or
writes exactly N, 3 N or Q N elements): both the same-name module functions
and the Lattices methods.  Runs on the CPU: the checks come before any
library call, on a wrapper object that holds no handle."""
import numpy as np
import pytest

import paper_2112_08926_amd as lbm


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


def test_module_functions_refuse_wrong_sizes():
    n = 64
    with pytest.raises(ValueError, match="flags"):
        lbm.lbm_set_boundaries(None, 0, np.zeros(n - 1, np.uint8), n)
    with pytest.raises(ValueError, match="rho"):
        lbm.lbm_set_rho_u(None, 0, n, rho=np.ones(n - 1))
    with pytest.raises(ValueError, match="u"):
        lbm.lbm_set_rho_u(None, 0, n, u=np.zeros(3 * n + 3))
    with pytest.raises(ValueError, match="u_ref"):
        lbm.lbm_diagnostics(None, 0, n, np.zeros(2 * n))
    with pytest.raises(ValueError, match="codes"):
        lbm.lbm_set_ddf(None, 0, np.zeros((19, n - 1), np.uint16), n, 19)
    with pytest.raises(ValueError, match="out"):
        lbm.lbm_get_ddf(None, 0, np.zeros((19, n + 1), np.uint16), n, 19)
    with pytest.raises(ValueError, match="out"):
        lbm.lbm_get_ddf(None, 0, np.zeros((19, 2 * n), np.uint16)[:, ::2], n, 19)   # not contiguous


def test_host_arrays_of_any_shape_of_the_right_size_are_taken():
    from paper_2112_08926_amd import _lib
    a = np.arange(24, dtype=np.int64).reshape(2, 3, 4)
    c = _lib._check_host(a, 24, np.float64, "x")
    assert c.dtype == np.float64 and c.flags.c_contiguous and np.array_equal(c, a.astype(np.float64))
    f = np.asfortranarray(np.arange(6.0).reshape(2, 3))
    assert np.array_equal(_lib._check_host(f, 6, np.float64, "x"), np.arange(6.0).reshape(2, 3))
