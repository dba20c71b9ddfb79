"""Host side of the PML operator in the native library (no GPU calls): the
one-sided tables and the Fornberg weights the kernels use, the spectrum
reading and the grid checks, against the pinned oracle."""
import numpy as np
import pytest

from oracle import pml
from paper_2401_16322_amd import expwave as ew


def test_surface_tables_match_the_oracle():
    d2, d1, dw = ew.expw_pml_surface_weights()
    assert np.array_equal(d2, np.array([[float(c) for c in r] for r in pml.SURFACE_D2]))
    assert np.array_equal(d1, np.array([[float(c) for c in r] for r in pml.SURFACE_D1]))
    # Fornberg in FP64 against the oracle's exact rational weights
    want = np.array([[float(c) for c in r] for r in pml.surface_dw_weights()])
    assert np.max(np.abs(dw - want)) <= 1e-13 * np.max(np.abs(want))


@pytest.mark.parametrize("cells,beta0", [(0, 0.0), (6, 150.0)])
def test_spectrum_rectangle_matches_the_oracle_reading(cells, beta0):
    g = pml.PMLGrid(40, 30, 10.0, abc_cells=cells, beta0=beta0)
    c2 = np.full(g.shape, 2500.0 ** 2)
    want = pml.spectrum_rectangle_pml(g, c2)
    got = ew.expw_pml_spectrum_rectangle(ew.make_pml_grid(40, 30, 10.0, ew.EXPW_F64, cells, beta0), 2500.0 ** 2)
    assert np.allclose(got, want, rtol=1e-14, atol=0.0)


@pytest.mark.parametrize("nx,ny,h,cells,beta0", [(10, 8, 1.0, 0, 0.0), (0, 20, 1.0, 0, 0.0),
                                                 (10, 20, 0.0, 0, 0.0), (10, 20, 1.0, -1, 0.0),
                                                 (10, 20, 1.0, 2, -5.0)])
def test_invalid_grids_are_rejected(nx, ny, h, cells, beta0):
    with pytest.raises(ew.ExpwError) as e:
        ew.expw_pml_workspace_size(ew.make_pml_grid(nx, ny, h, ew.EXPW_F32, cells, beta0), 8)
    assert e.value.status == ew.EXPW_EINVAL


def test_workspace_holds_three_states():
    g = ew.make_pml_grid(100, 50, 5.0, ew.EXPW_F64, 4, 100.0)
    assert ew.expw_pml_workspace_size(g, 8) >= 3 * 4 * 100 * 50 * 8
