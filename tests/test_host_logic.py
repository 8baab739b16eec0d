"""Host-side logic that needs no GPU: the autotuner's candidate forms and shape buckets."""
from paper_2506_23928_amd import tvmc
from paper_2506_23928_amd.autotune import bucket, candidates


def test_candidates_are_result_preserving_forms():
    # Jastrow, M <= N_s: two solver layouts x two exact S-build precisions
    c = candidates(tvmc.JASTROW, 36, 1024)
    assert len(c) == 4 and {x["solver"] for x in c} == {tvmc.SOLVER_ONE_GROUP, tvmc.SOLVER_MULTI_GROUP}
    assert {x["precision"] for x in c} == {tvmc.PREC_MFMA, tvmc.PREC_FP64}
    # M > N_s adds the sample-space solve (the push-through identity)
    c = candidates(tvmc.JASTROW, 2080, 2048)
    assert tvmc.SOLVER_SAMPLE_SPACE in {x["solver"] for x in c} and len(c) == 6
    # RBM: its BF16-split S is not bit-equal to the FP64 one, so precision is never a candidate
    c = candidates(tvmc.RBM, 4224, 8192)
    assert all("precision" not in x for x in c) and len(c) == 2
    # LJPHd and the SNR solve stay in parameter space
    assert tvmc.SOLVER_SAMPLE_SPACE not in {x["solver"] for x in candidates(tvmc.LJPH, 300, 256)}
    assert tvmc.SOLVER_SAMPLE_SPACE not in {x["solver"] for x in candidates(tvmc.JASTROW, 300, 256, tvmc.REG_SNR)}


def test_buckets_separate_shapes():
    a = bucket(0, 64, 0, 2080, 256, 4096, 64)
    assert a == bucket(0, 64, 0, 2080, 256, 4096, 64)
    assert len({a, bucket(0, 64, 0, 2080, 128, 4096, 64), bucket(0, 64, 0, 2080, 256, 2048, 64),
                bucket(1, 64, 64, 4224, 256, 4096, 64), bucket(0, 64, 0, 2080, 256, 4096, 64, 1)}) == 5
