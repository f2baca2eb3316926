"""Seeded generators: determinism, pattern structure and sizes."""
import numpy as np

from synth import configs
from synth.silicon import si_bulk, si_slab_001


def test_si64_pattern():
    c = configs.si64()
    s = c["system"]
    assert s.n == 256 and s.nnzb == 1088
    assert np.all(np.diff(s.rowptr) == 17)
    for i in range(s.nb):
        cols = s.colidx[s.rowptr[i]:s.rowptr[i + 1]]
        assert np.all(np.diff(cols) > 0) and i in cols
    m = s.mirror()
    np.testing.assert_array_equal(s.ang[m], np.transpose(s.ang, (0, 2, 1)))
    np.testing.assert_array_equal(s.trans[m], -s.trans)
    np.testing.assert_array_equal(c["rhs"], np.arange(8))


def test_determinism():
    a = configs.si_small(seed=5)["system"]
    b = configs.si_small(seed=5)["system"]
    np.testing.assert_array_equal(a.positions, b.positions)
    np.testing.assert_array_equal(a.ang, b.ang)
    c = configs.si_small(seed=6)["system"]
    assert not np.array_equal(a.ang, c.ang)


def test_shell_distances():
    s = si_bulk((2, 2, 2))
    rows = s.block_rows()
    d = s.positions[s.colidx] + s.trans - s.positions[rows]
    r = np.linalg.norm(d, axis=1)
    off = rows != s.colidx
    vals = np.unique(np.round(r[off], 3))
    np.testing.assert_allclose(vals, [2.352, 3.840], atol=2e-3)


def test_slab_dimers():
    s = si_slab_001((2, 2, 4))
    assert s.meta["n_dimer_atoms"] > 0
    assert np.isinf(s.box[2])


def test_water_small():
    c = configs.water_small(n_mol=32)
    s = c["system"]
    assert s.block == 6 and s.n == 192
    m = s.mirror()
    np.testing.assert_array_equal(s.ang[m], np.transpose(s.ang, (0, 2, 1)))
