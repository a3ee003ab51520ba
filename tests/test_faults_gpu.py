"""Error paths under injected device-allocation failures
(sal_debug_fail_allocation): every allocation point of context creation,
surface-set creation, labeling and refinement fails once in turn; the call
that meets it reports out of memory, a refine round that fails leaves the
mesh as it was, and after disarming, the same objects (or new ones) give the
results of a run without failures."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
import paper_2203_10000_amd as sal  # noqa: E402

pytestmark = pytest.mark.gpu

OOM, DEVICE = 4, 5


@pytest.fixture(scope="module")
def case():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cfg = synth.config_small("head", cells=8, subdiv=2)
    rng = np.random.default_rng(71)
    pts = synth.uniform_box(rng, 20000, -100, 100)
    return cfg, pts


def _run(cfg, pts, rule, state):
    """The sequence, resumable: creates what `state` lacks, then labels and
    refines.  Raises SalError at the first failure."""
    if "ctx" not in state:
        state["ctx"] = sal.Context(0)
    ctx = state["ctx"]
    if "ss" not in state:
        state["ss"] = sal.SurfaceSet(ctx, cfg.surfaces)
    if "labels" not in state:
        dev = torch.from_numpy(pts).to("cuda:0").contiguous()
        lab, _, _ = sal.label_points(ctx, state["ss"], dev)
        state["labels"] = lab.cpu().numpy()
    lat = cfg.lattice
    if "mesh" not in state:
        state["mesh"] = sal.TetMesh(ctx, lat.origin, lat.h, lat.cells)
    mesh = state["mesh"]
    while mesh.size()[1] < 2:
        mesh.refine_relabel(state["ss"], 1, rule=rule)
    e = mesh.export(keys=True, labels=True, centroids=False)
    return state["labels"], e["keys"].cpu().numpy(), e["labels"].cpu().numpy()


@pytest.mark.parametrize("rule", ["centroid", "four_nodes"])
def test_every_allocation_failure_is_reported_and_recoverable(case, rule):
    cfg, pts = case
    want = _run(cfg, pts, rule, {})
    failures = 0
    for k in range(1, 200):
        state = {}
        sal.lib().sal_debug_fail_allocation(k)
        try:
            got = _run(cfg, pts, rule, state)
            hit = False
        except sal.SalError as e:
            hit = True
            assert e.status in (OOM, DEVICE), (k, e.status, str(e))
            if "mesh" in state and "labels" in state:
                # a failed refine round changes nothing: leaves == N0 + 7 x split
                n, lv = state["mesh"].size()
                keys = state["mesh"].export(keys=True, labels=False, centroids=False)["keys"]
                assert len(keys) == n
        finally:
            sal.lib().sal_debug_fail_allocation(0)
        if not hit:
            # k is past the last allocation of the whole sequence
            assert failures > 0
            for a, b in zip(got, want):
                assert np.array_equal(a, b)
            break
        failures += 1
        got = _run(cfg, pts, rule, state)       # the same objects, disarmed
        for a, b in zip(got, want):
            assert np.array_equal(a, b), k
    else:
        pytest.fail("the sequence kept failing")
    assert failures >= 8
