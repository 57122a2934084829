"""The seeded input generators: the random smooth state against its plain
definition, and the bounds its docstring states."""
import math

import numpy as np

import workloads as wl


def test_random_smooth_matches_its_definition():
    """Sum over modes k of a_k cos(2 pi k.x / L) + b_k sin(2 pi k.x / L),
    written out mode by mode, against the chunked product evaluation."""
    for dim in (2, 3):
        st = wl.RandomSmooth(dim, 2.0 * math.pi, 7)
        x = np.random.default_rng(1).uniform(-1.0, 7.0, size=(3000, dim))
        ref = np.zeros((x.shape[0], dim + 2))
        for j, k in enumerate(st._modes):
            arg = 2.0 * math.pi / st.L * (x @ k)
            for c, cs in enumerate(st._coef):
                ref[:, c] += cs[j, 0] * np.cos(arg) + cs[j, 1] * np.sin(arg)
        assert np.abs(st._phis(x, chunk=777) - ref).max() < 1e-14
        # |Phi| <= 1 by the normalisation: density and pressure in [0.8, 1.2]
        u = st(x)
        assert u[:, 0].min() >= 0.8 - 1e-15 and u[:, 0].max() <= 1.2 + 1e-15
