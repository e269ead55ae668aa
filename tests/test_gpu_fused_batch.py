"""GPU parity of the fused convolution, the fused permute/scale and the
batched persistent launch (plain and captured in a HIP graph) against the
CPU oracle, bit for bit."""
import numpy as np
import pytest
import torch

import ne_synth

pytestmark = pytest.mark.gpu

DEV = "cuda"


@pytest.fixture(scope="module")
def ne():
    import paper_1604_04740_amd as ne
    ne.lib()
    return ne


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _h(t):
    return t.cpu().numpy()


def _bits(words, count):
    w = np.asarray(words).astype(np.int64) & 0xFFFFFFFF
    bits = (w[..., None] >> np.arange(32)) & 1
    return bits.reshape(*w.shape[:-1], -1)[..., :count].astype(bool)


@pytest.mark.parametrize("M,N", [(3, 1), (3, 300), (4, 1000), (3, 16384), (5, 257), (8, 513)])
def test_circconv_fused(ne, orc, M, N):
    c, g = ne_synth.conv_streams(1300 + M + N, M, N, -1024, 1024, -64, 64)
    p = ne.ne_params_default(M)
    for r in sorted({0, M - 1}):
        p.r_check = r
        ref = orc.conv_pipeline(c, g.astype(np.int64), r=r)
        for cdt in (np.int32, np.int64):
            dh, fl, nb = ne.ne_circconv_fused(_t(c.astype(cdt)), _t(g), p, c_bits=11)
            assert np.array_equal(_h(dh), ref["dhat"]), (r, cdt)
            assert int(nb.item()) == 0 and not _bits(_h(fl), N).any()
    dh32, _, _ = ne.ne_circconv_fused(_t(c.astype(np.int32)), _t(g), p, c_bits=11,
                                      out_dtype=torch.int32)
    assert np.array_equal(_h(dh32), ref["dhat"].astype(np.int32))
    # without a workspace: one workgroup per block of 1024 outputs
    dh, fl, nb = ne.ne_circconv_fused(_t(c), _t(g), p, c_bits=11, workspace=None)
    assert np.array_equal(_h(dh), ref["dhat"]) and int(nb.item()) == 0


@pytest.mark.parametrize("M,N,cdt,bits", [(6, 2500, np.int8, 8), (3, 700, np.int32, 20),
                                          (4, 1024, np.int64, 14)])
def test_circconv_fused_digit_counts(ne, orc, M, N, cdt, bits):
    """One, two and three int8 digits per input value; full and ragged blocks."""
    lo = -(1 << (bits - 1))
    c = ne_synth.uniform_int(1350 + M + N, 1, (M, N), lo, -lo)
    g = ne_synth.uniform_int(1350 + M + N, 2, (N,), -128, 128).astype(np.int8)
    p = ne.ne_params_default(M)
    p.r_check = M - 1
    ref = orc.conv_pipeline(c, g.astype(np.int64), r=M - 1)
    dh, fl, nb = ne.ne_circconv_fused(_t(c.astype(cdt)), _t(g), p, c_bits=bits)
    assert np.array_equal(_h(dh), ref["dhat"])
    assert int(nb.item()) == 0 and not _bits(_h(fl), N).any()


def test_circconv_fused_range_check(ne):
    p = ne.ne_params_default(8)  # l = 8, k = 8: D = 127 * 2^48
    c = torch.zeros((8, 16), dtype=torch.int64, device=DEV)
    g = torch.zeros((16,), dtype=torch.int8, device=DEV)
    with pytest.raises(ne.NEError) as e:
        ne.ne_circconv_fused(c, g, p, c_bits=50)
    assert e.value.code == -2


@pytest.mark.parametrize("M,N", [(3, 1), (3, 1000), (5, 4099), (8, 70000)])
def test_permute_scale_fused(ne, orc, M, N):
    c, perm, s, a = ne_synth.perm_scale_streams(1400 + M + N, M, N, -128, 128)
    p = ne.ne_params_default(M)
    for r in sorted({0, M - 2}):
        p.r_check = r
        ref = orc.permute_scale_pipeline(c, perm, s, a, r=r)
        dh, fl, nb = ne.ne_permute_scale_fused(_t(c.astype(np.int8)), _t(perm.astype(np.int32)),
                                               _t(s), _t(a), p)
        assert np.array_equal(_h(dh), ref["dhat"]) and int(nb.item()) == 0
        assert not _bits(_h(fl), N).any()
    dh, fl, nb = ne.ne_permute_scale_fused(_t(c), _t(perm.astype(np.int32)), None, None, p)
    ref2 = orc.permute_scale_pipeline(c, perm, None, None, r=p.r_check)
    assert np.array_equal(_h(dh), ref2["dhat"])
    # direct gather from c (no row copy)
    for cdt in (np.int8, np.int32):
        dh, fl, nb = ne.ne_permute_scale_fused(_t(c.astype(cdt)), _t(perm.astype(np.int32)),
                                               _t(s), _t(a), p, workspace=None)
        ref3 = orc.permute_scale_pipeline(c, perm, s, a, r=p.r_check)
        assert np.array_equal(_h(dh), ref3["dhat"]) and int(nb.item()) == 0


def _problems(ne, recipe):
    probs = []
    for i, q in enumerate(recipe):
        r = i % q["M"]
        if q["op"] == 0:
            probs.append(ne.Problem(ne.NE_OP_GEMM, _t(q["c"]), _t(np.ascontiguousarray(q["G"].T)),
                                    r_check=r, out_dtype=torch.int64 if i % 2 else torch.int32))
        elif q["op"] == 1:
            probs.append(ne.Problem(ne.NE_OP_CONV, _t(q["c"]), _t(q["g"]), r_check=r,
                                    out_dtype=torch.int64))
        else:
            probs.append(ne.Problem(ne.NE_OP_PERM, _t(q["c"]), None, perm=_t(q["perm"]),
                                    scale=_t(q["scale"]), add=_t(q["add"]), r_check=r,
                                    out_dtype=torch.int64))
    return probs


def _expected(orc, q, r):
    if q["op"] == 0:
        return orc.gemm_pipeline(q["c"], q["G"], r=r)["dhat"]
    if q["op"] == 1:
        return orc.conv_pipeline(q["c"].astype(np.int64), q["g"].astype(np.int64), r=r)["dhat"]
    return orc.permute_scale_pipeline(q["c"].astype(np.int64), q["perm"], q["scale"], q["add"],
                                      r=r)["dhat"]


def _check_all(probs, recipe, orc, expected=None):
    for i, (pb, q) in enumerate(zip(probs, recipe)):
        exp = expected[i] if expected is not None else _expected(orc, q, i % q["M"])
        got = _h(pb.d_hat).astype(np.int64)
        if pb.out_dtype == torch.int32:
            exp = exp.astype(np.int32).astype(np.int64)
        assert np.array_equal(got, exp), (i, q["op"], q["M"])
        assert int(pb.n_bad.item()) == 0, i


@pytest.fixture(scope="module")
def small_batch(ne, orc):
    recipe = ne_synth.batch_recipe(1500, 40, 40, 300)
    expected = [_expected(orc, q, i % q["M"]) for i, q in enumerate(recipe)]
    return recipe, expected


def test_batch_mixed_problems(ne, orc, small_batch):
    recipe, expected = small_batch
    assert {q["op"] for q in recipe} == {0, 1, 2}
    probs = _problems(ne, recipe)
    b = ne.Batch(probs)
    assert b.items > len(probs)
    b.run()
    torch.cuda.synchronize()
    _check_all(probs, recipe, orc, expected)
    # a second run of the same plan (the work counter is reset by the launch)
    for pb in probs:
        pb.d_hat.zero_()
        pb.n_bad.zero_()
    b.run()
    torch.cuda.synchronize()
    _check_all(probs, recipe, orc, expected)


def test_batch_in_hip_graph(ne, orc, small_batch):
    """Capture ne_batch_run in a graph; replay three times with eager work
    (clearing the outputs) between replays; every replay is exact."""
    recipe, expected = small_batch
    probs = _problems(ne, recipe)
    b = ne.Batch(probs)
    b.run()  # warm-up outside capture
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            b.run()
    torch.cuda.synchronize()
    for rep in range(3):
        for pb in probs:
            pb.d_hat.fill_(-7)
            pb.n_bad.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        _check_all(probs, recipe, orc, expected)


def test_batch_autotune_and_tuned_plan(ne, orc, small_batch):
    recipe, expected = small_batch
    probs = _problems(ne, recipe)
    t = ne.ne_batch_autotune(probs, reps=2)
    for m in range(6):
        for c in range(3):
            assert t.gemm_bn[m][c] in (128, 256)
            assert t.perm_chunk[m][c] % 64 == 0
    b = ne.Batch(probs, t)
    for pb in probs:
        pb.n_bad.zero_()
    b.run()
    torch.cuda.synchronize()
    _check_all(probs, recipe, orc, expected)


def test_batch_rejects_bad_problems(ne):
    c = torch.zeros((3, 4, 20), dtype=torch.int8, device=DEV)  # K % 16 != 0
    g = torch.zeros((4, 20), dtype=torch.int8, device=DEV)
    with pytest.raises(ne.NEError) as e:
        ne.Batch([ne.Problem(ne.NE_OP_GEMM, c, g)])
    assert e.value.code == -4
    c9 = torch.zeros((9, 64), dtype=torch.int8, device=DEV)
    with pytest.raises(ne.NEError):
        ne.Batch([ne.Problem(ne.NE_OP_CONV, c9, torch.zeros(64, dtype=torch.int8, device=DEV))])
