"""Short runs of the robustness driver (Sec. 7.5): the entropy-conservative
scheme conserves the entropy integral to rounding on the Taylor-Green vortex
at Ma 0.1, and the entropy-stable scheme never increases it on the
Kelvin-Helmholtz instability; both stay admissible over the interval."""
import pytest
import torch

import workloads as wl
from tests.parity_util import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()


def test_tgv_entropy_conservative_short():
    from paper_2312_07874_amd import robustness as RB
    r = RB.run(wl.tgv_tet_mach(4, 4, 0.1, dissipation=0), 0.5, snapshots=20, log=log)
    assert r["completed"]
    S0 = r["history"][0][1]
    # rounding of the entropy integral accumulated over the steps
    assert abs(r["entropy_change"]) <= 1e-10 * abs(S0), r["entropy_change"]


def test_khi_entropy_stable_short():
    from paper_2312_07874_amd import robustness as RB
    r = RB.run(wl.khi_tri(16, 4, dissipation=1), 1.0, snapshots=20, log=log)
    assert r["completed"]
    assert r["entropy_nonincreasing"]
    assert r["max_entropy_rate"] <= 1e-12 * abs(r["history"][0][1])
