"""The entry point that allocates nothing (srp_eval_batch_noalloc), through
the C ABI, against srp_eval_batch on the same items: bitwise the same result
records on two calls in a row (the second with a smaller batch, so the fixed
workspace still holds the first call's contents), and a batch too large for
the fixed workspace rejected with an error."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def srp():
    import torch
    assert torch.cuda.is_available()
    import paper_2608_07307_amd as m
    return m


def _batch(srp, scenes, count, seed):
    """Mixed scenes, grid sizes (ragged ones included), bounce counts, diffuse
    fans, per-item angles or the scene's current ones."""
    entries = []
    for k in range(count):
        sc, m = scenes[0] if k % 3 == 0 else scenes[1]
        B = k % 3
        K = 4 if (k % 4 == 1 and B > 0) else 0
        n = [64, 100, 128, 37, 256][k % 5]
        ang = np.full(m.n_dof, 0.07 * (k % 5) - 0.1) if k % 2 == 0 else None
        entries.append((sc, ang, srp.params(synth.random_dirs(seed + k)[0], n, B, diffuse=K)))
    return entries


def test_noalloc_matches_eval_batch(srp):
    import torch
    m1, m2 = synth.box_wing(), synth.procedural_sized(22, 4000)
    scenes = [(srp.Scene(m1), m1), (srp.Scene(m2), m2)]
    stream = torch.cuda.current_stream()
    for count, seed in ((14, 7100), (3, 7200)):
        entries = _batch(srp, scenes, count, seed)
        ref = srp.results_to_numpy(srp.eval_batch(entries)).copy()
        out = torch.full((count * srp.RESULT_DTYPE.itemsize,), 0xAB, dtype=torch.uint8, device="cuda")
        srp.eval_batch_noalloc(entries, out, stream)
        got = srp.results_to_numpy(out)
        print(f"no-alloc batch of {count}: status {got['status'].tolist()}, hits {got['n_hits'].tolist()}",
              flush=True)
        assert (got["status"] == 0).all() and (got["n_hits"] > 0).all()
        assert got.tobytes() == ref.tobytes()
    # one 8192^2 evaluation needs 64 MiB of patch partials alone: rejected, not split
    with pytest.raises(srp.SrpError, match="fixed workspace"):
        srp.eval_batch_noalloc([(scenes[1][0], None, srp.params((0.0, 0.0, 1.0), 8192, 0))])
    for sc, _ in scenes:
        sc.close()
