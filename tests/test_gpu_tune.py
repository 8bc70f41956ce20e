"""The launch-shape autotuner: every candidate gives the same bytes (it
raises otherwise), the fastest is kept in force, and the output under the
tuned shape equals the oracle's."""
import numpy as np
import pytest

from gpu_util import require_gpu, to_np_u32, to_np_u64

pytestmark = pytest.mark.gpu


def test_tune_picks_a_candidate_and_keeps_bits(kgref):
    import torch
    kg = require_gpu()
    from paper_1710_07565_amd import tune
    insts = [kg.Instance(3000, kg.GNM, False, 200000, 0.0, kg.instance_seed(4, 0), 9),
             kg.Instance(2**14, kg.GNP, True, 0, 8.0 / (2**14 - 1), kg.instance_seed(4, 1), 5),
             kg.Instance(700, kg.GNM, True, 300000, 0.0, kg.instance_seed(4, 2), 3)]
    try:
        res = tune.tune(insts, sample_waves=(0, 2), plan_waves=(0, 3), leaf_cap=(0, 256), reps=1)
        assert len(res["table"]) == 8
        best = res["best"]
        assert best in res["table"]
        assert kg.get_option(kg._lib.KG_OPT_SAMPLE_WAVES) == best["sample_waves"]
        assert kg.get_option(kg._lib.KG_OPT_PLAN_WAVES) == best["plan_waves"]
        arena, offs = kg.batch(insts)
        torch.cuda.synchronize()
        A, O = to_np_u32(arena), to_np_u64(offs)
        for i, I in enumerate(insts):
            want = kgref.generate(kgref.inst(I.n, m=I.m, p=I.p, directed=I.directed, seed=I.seed,
                                             chunks=I.chunks, model=I.model))
            assert np.array_equal(A[O[i]:O[i + 1]], want), i
    finally:
        for o in (kg._lib.KG_OPT_SAMPLE_WAVES, kg._lib.KG_OPT_PLAN_WAVES, kg._lib.KG_OPT_LEAF_CAP):
            kg.set_option(o, 0)
