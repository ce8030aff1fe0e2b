"""The 12 spin-colour point sources follow the index idx = ic + Nc*id of the
propagator loop in the paper's Fig. 1 listing (tests/golden/spin_colour_index.txt)."""
import os

import numpy as np

from lattice_inputs import point_sources

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "spin_colour_index.txt")


def test_point_source_index_convention():
    rows = [tuple(int(v) for v in ln.split()) for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 12
    src = point_sources((2, 2, 2, 2))
    for idx, spin, colour in rows:
        nz = np.argwhere(src[idx] != 0)
        assert nz.tolist() == [[0, 0, 0, 0, spin, colour]]
        assert src[idx][0, 0, 0, 0, spin, colour] == 1.0
