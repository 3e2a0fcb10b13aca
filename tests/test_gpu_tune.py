"""SpMV schedules and the autotuner: every schedule gives bitwise the same output (each row is
evaluated by one lane in the same order whatever workgroup runs it), and the autotuner keeps
one of them."""
import numpy as np
import pytest

import workloads as wl

from _util import c2_keys, c3_parts, heavy_hex_small, say

torch = pytest.importorskip("torch")
qsd = pytest.importorskip("paper_2603_18731_amd")

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    qsd.lib()


def _ham(keys, tl):
    return qsd.SubspaceHamiltonian(qsd.Subspace(keys, tl.n_qubits), qsd.operator_from_termlist(tl))


@pytest.mark.parametrize("case", ["xxz", "fermi", "heavyhex"])
def test_schedules_bitwise(case):
    if case == "xxz":
        H = _ham(c2_keys(50_000), wl.xxz_grid_6x6())
    elif case == "fermi":
        ops, keys = c3_parts(90, 90)
        H = _ham(keys, ops)
    else:
        tl, keys = heavy_hex_small(30_001)
        H = _ham(keys, tl)
    rng = np.random.default_rng(3)
    x = torch.from_numpy(rng.standard_normal((H.N, 3))).cuda()
    outs = []
    for sched in (0, qsd.SCHED_XCD_REMAP):
        H.schedule = sched
        outs.append(H.matvec(x))
    torch.cuda.synchronize()
    say(case, "N", H.N)
    assert torch.equal(outs[0], outs[1])
    r = H.autotune(nvec=1, reps=2)
    say(case, "autotune ->", r)
    assert r["schedule"] in (0, qsd.SCHED_XCD_REMAP) and H.schedule == r["schedule"] and r["ms"] > 0
    assert r["max_load"] in (0.0625, 0.125, 0.25, 0.5) and H.subspace.capacity == r["capacity"]
    assert torch.equal(H.matvec(x), outs[0])  # a rebuilt table gives the same output
    keys_before = H.subspace.keys()
    for load in (0.5, 0.03):
        H.subspace.rehash(load)
        assert torch.equal(H.matvec(x), outs[0])
        assert torch.equal(H.subspace.lookup(keys_before), torch.arange(H.N, device="cuda"))
    with pytest.raises(qsd.QsdError, match="INVALID_ARG"):
        H.schedule = 0x80
