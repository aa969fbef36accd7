"""Captured forward launches of one patch per chunk (repeated single
evaluations, small batch plans) hand out their patches heaviest first, in the
order the previous launch measured.  The order only decides which wave traces
a patch and when: every patch writes its own partial slot and the reduction
sums the slots in a fixed order (Sec. 4.3: one ray per pixel, sums on the
GPU), so results must be bitwise equal across replays, across sequences of
different attitudes and to the direct batch path, which keeps image order."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

FIELDS = ("force", "torque", "n_rays", "n_hits", "n_secondary", "n_secondary_hits", "n_box_tests",
          "n_tri_tests", "status", "n_clamped")


@pytest.fixture(scope="module")
def srp():
    import torch
    assert torch.cuda.is_available()
    import paper_2608_07307_amd as m
    return m


def _same(a, b, ctx):
    for f in FIELDS:
        assert np.array_equal(np.asarray(a[f]), np.asarray(b[f])), (ctx, f, a[f], b[f])


@pytest.mark.parametrize("case,n,bounces,count,diffuse", [
    ("plain", 256, 2, False, 0),
    ("counting", 96, 2, True, 0),
    ("diffuse", 64, 2, False, 8),
])
def test_repeated_single_evaluations_match_the_direct_path(srp, case, n, bounces, count, diffuse):
    mesh = synth.procedural_sized(31, 4000)
    sc = srp.Scene(mesh)
    ang = np.random.default_rng(77).uniform(-1.0, 1.0, mesh.n_dof)
    sc.set_angles(ang)
    suns = synth.random_dirs(8100 + n, 3)
    print(f"{case}: {mesh.n_tris} tris, n {n}, B {bounces}, diffuse {diffuse}", flush=True)
    ref = []
    for k in range(3):
        p = srp.params(suns[k], n, bounces, count=count, diffuse=diffuse)
        ref.append(srp.results_to_numpy(srp.eval_batch([(sc, ang, p)]))[0])
    assert ref[0]["n_hits"] > 0
    # attitudes 0, 1, 2, 0, ...: each call replays the scene's captured
    # evaluation with the order the previous call (another attitude) measured
    for rep in range(3):
        for k in (0, 1, 2, 0):
            r = srp.eval(sc, suns[k], n, bounces=bounces, count=count, diffuse=diffuse)
            _same(r, ref[k], (case, rep, k))


def test_batch_plan_replays_match_the_direct_path(srp):
    import torch
    meshes = [synth.box_wing(), synth.procedural_sized(33, 3000)]
    scenes = [srp.Scene(m) for m in meshes]
    suns = synth.random_dirs(8200, 6)
    entries = [(scenes[k % 2], None, srp.params(suns[k], [48, 80, 128][k % 3], 1 + k % 2)) for k in range(6)]
    ref = srp.results_to_numpy(srp.eval_batch(entries))
    plan = srp.Plan(entries)
    for rep in range(4):
        out = srp.results_to_numpy(plan.launch())
        torch.cuda.synchronize()
        assert out.tobytes() == ref.tobytes(), rep
    entries2 = [(sc, a, srp.params(suns[(k + 3) % 6], n, b)) for k, (sc, a, p) in enumerate(entries)
                for n, b in [(p.n, p.bounces)]]
    plan.update(entries2)
    for rep in range(2):
        out2 = srp.results_to_numpy(plan.launch())
        torch.cuda.synchronize()
        assert out2.tobytes() == srp.results_to_numpy(srp.eval_batch(entries2)).tobytes(), rep
    plan.close()
