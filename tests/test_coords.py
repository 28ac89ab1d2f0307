"""The package's (f, alpha) coordinate helpers against the oracle's maps (CPU only; numpy on both sides)."""
import numpy as np
import pytest

import paper_2506_18003_amd as scd
from oracle import scd_oracle as O


@pytest.mark.parametrize("Np,N", [(16, 1024), (64, 1 << 12), (256, 2048)])
def test_ssca_coords_equal_oracle(Np, N):
    """Pinned on the oracle side against the Eq. (2) demodulate frequencies."""
    for a, b in zip(scd.ssca_coords(Np, N), O.ssca_coords(Np, N)):
        assert np.array_equal(np.broadcast_to(a, b.shape), b)


@pytest.mark.parametrize("Np,L,P", [(16, 4, 32), (256, 64, 32), (32, 8, 64)])
def test_fam_coords_equal_oracle(Np, L, P):
    """Pinned on the oracle side by the two-tone cycle-frequency test."""
    for a, b in zip(scd.fam_coords(Np, L, P), O.fam_coords(Np, L, P)):
        assert np.array_equal(np.broadcast_to(a, b.shape), b)
