"""The work-shape autotuner: its size buckets and cache (CPU), and on the GPU a
sweep over a few candidate shapes that picks one per pass, records it, and
whose shapes give the same results bitwise as the library defaults."""
import numpy as np
import pytest

from paper_1803_09652_amd import autotune as at


def test_bucket_key_groups_batches_by_powers_of_two():
    a = at.bucket_key([0, 2500, 5000], "fp32")
    assert a == at.bucket_key([0, 2400, 4900], "fp32")          # same powers of two
    assert a != at.bucket_key([0, 2500, 5000], "fp64")          # precision is part of the key
    assert a != at.bucket_key([0, 2500, 5000, 7500], "fp32")    # more systems
    assert a != at.bucket_key([0, 5000, 10000], "fp32")         # larger systems
    assert at.bucket_key([0], "fp32").startswith("fp32:")       # empty batch still keys


def test_cache_round_trip(tmp_path, monkeypatch):
    path = tmp_path / "tuning.json"
    monkeypatch.setenv("GBMC_TUNING_CACHE", str(path))
    off = [0, 900, 1233]
    assert at.lookup(off, "fp32") is None
    at._save_cache({at.bucket_key(off, "fp32"): {"j_blocks_per_item": [1, 2, 4],
                                                "waves_per_group": [2, 4, 8], "pair_ms": 1.0}})
    assert at.lookup(off, "fp32") == ((1, 2, 4), (2, 4, 8))
    assert at.lookup(off, "fp64") is None
    path.write_text("not json")
    assert at.lookup(off, "fp32") is None                        # a broken cache is ignored


@pytest.mark.gpu
def test_tune_picks_a_candidate_per_pass_and_keeps_results(tmp_path, monkeypatch):
    import torch
    import synth
    from gpu_common import build, gpu_eval, params_pair
    monkeypatch.setenv("GBMC_TUNING_CACHE", str(tmp_path / "tuning.json"))
    systems = [synth.make_system(31, 700, 10.0), synth.make_system(32, 1500, 14.0)]
    batch = synth.make_batch(systems)
    cands = [(1, 1), (2, 4), (4, 2)]
    r = at.tune(batch, "fp32", candidates=cands, reps=2)
    jbs, wvs = r["best"]
    for k in range(3):
        assert (jbs[k], wvs[k]) in cands
    assert set(r["ms"]) == {f"{j}x{w}" for j, w in cands}
    assert all(v > 0 for v in r["ms"].values())
    # each pass takes its own best shape (medians per kernel, so within noise of any one shape)
    assert r["pair_ms"] <= 1.05 * min(r["ms"].values())
    assert at.lookup(batch.atom_offset, "fp32") == (tuple(jbs), tuple(wvs))
    p_gpu, _ = params_pair()
    _, _, plan_d, atoms_d = build(systems, "fp32")
    _, _, plan_t, atoms_t = build(systems, "fp32", j_blocks=jbs, waves=wvs)
    a, b = gpu_eval(plan_d, atoms_d, p_gpu), gpu_eval(plan_t, atoms_t, p_gpu)
    torch.cuda.synchronize()
    for k in ("R", "Ec", "Egb", "force", "dEdq", "dEdrho"):
        assert np.array_equal(a[k], b[k]), k
