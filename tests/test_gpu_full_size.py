"""GPU parity at the benchmark workloads' full sizes, in the launch
configurations bench.py times: sampled outputs against the oracle computed a
row (or a problem) at a time, plus the properties that hold at any size
(no flags on clean data, exactly the injected positions flagged, exact
recovery)."""
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


def _flag_bits_at(fl, pos, N):
    w = fl.cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    return (w[pos // N, (pos % N) // 32] >> ((pos % N) % 32)) & 1


def test_gemm_m4_4096_sampled(ne, orc):
    """The headline workload (M = 4, 4096^3, U[-127,127]), int32 d_hat and
    row-padded flags as timed: sampled rows equal the oracle's pipeline on
    those rows, the whole output equals the plain GEMM of the same streams,
    and nothing is flagged."""
    M, n = 4, 4096
    c, G = ne_synth.gemm_streams(ne_synth.BASE_SEED + 2, M, n, n, n, -127, 128)
    c_d = torch.from_numpy(c).to(DEV)
    Gt = torch.from_numpy(np.ascontiguousarray(G.T)).to(DEV)
    p = ne.ne_params_default(M)
    out = torch.empty((M, n, n), dtype=torch.int32, device=DEV)
    fl = torch.empty((n, n // 32), dtype=torch.int32, device=DEV)
    nb = torch.zeros((1,), dtype=torch.int64, device=DEV)
    ne.ne_gemm_fused(c_d, Gt, p, out=out, flags=fl, n_bad=nb)
    assert int(nb.item()) == 0 and int(fl.abs().sum().item()) == 0
    plain = ne.ne_plain_gemm_i8(c_d.reshape(M * n, n), Gt)
    assert torch.equal(plain.reshape(M, n, n), out)
    del plain
    rows = [0, 1, 2047, 4095] + list(ne_synth.uniform_int(5, 1, (3,), 0, n))
    got = out.cpu().numpy()
    for r in rows:
        ref = orc.gemm_pipeline(c[:, r:r + 1, :], G)
        assert ref["n_bad"] == 0
        assert np.array_equal(got[:, r, :], ref["dhat"][:, 0, :].astype(np.int32)), r


def test_stress_m3_8192_sampled(ne, orc):
    """The fault-stress workload (M = 3, 8192^3): sampled rows against the
    oracle; single-bit flips at a 1e-6 per-word rate in one stream are
    flagged exactly where injected; a fail-stop loss of any stream is
    recovered exactly from the other two."""
    M, n = 3, 8192
    seed = ne_synth.BASE_SEED + 4
    c, G = ne_synth.gemm_streams(seed, M, n, n, n, -127, 128)
    c_d = torch.from_numpy(c).to(DEV)
    Gt = torch.from_numpy(np.ascontiguousarray(G.T)).to(DEV)
    p = ne.ne_params_default(M)
    clean = torch.empty((M, n, n), dtype=torch.int32, device=DEV)
    fl = torch.empty((n, n // 32), dtype=torch.int32, device=DEV)
    nb = torch.zeros((1,), dtype=torch.int64, device=DEV)
    ne.ne_gemm_fused(c_d, Gt, p, out=clean, flags=fl, n_bad=nb)
    assert int(nb.item()) == 0
    got = clean[:, [0, 4321, 8191], :].cpu().numpy()
    for i, r in enumerate([0, 4321, 8191]):
        ref = orc.gemm_pipeline(c[:, r:r + 1, :], G)
        assert np.array_equal(got[:, i, :], ref["dhat"][:, 0, :].astype(np.int32)), r
    del got
    words = n * n
    for run in range(2):
        key = seed * 7919 + run
        stream = int(ne_synth.uniform_int(key, 1, (1,), 0, M)[0])
        gaps = np.random.default_rng(key).geometric(1e-6, size=int(words * 3e-6) + 16)
        pos = np.cumsum(gaps) - 1
        pos = pos[pos < words].astype(np.int64)
        bits = ne_synth.uniform_int(key, 2, (pos.size,), 0, 64).astype(np.uint64)
        mask = (np.uint64(1) << bits).view(np.int64)
        inj = ne.Inject(torch.from_numpy(pos).to(DEV),
                        torch.full((pos.size,), stream, dtype=torch.int32, device=DEV),
                        torch.from_numpy(mask).to(DEV))
        out = torch.empty_like(clean)
        nb.zero_()
        ne.ne_gemm_fused(c_d, Gt, p, out=out, flags=fl, n_bad=nb, inject=inj)
        assert pos.size > 0
        assert _flag_bits_at(fl, pos, n).all()
        assert int(nb.item()) == pos.size
        del out
    eps = ne.ne_entangle(c_d, p)
    delta = ne.ne_lsb_gemm(eps, 24, Gt, p)
    del eps
    for lost in range(M):
        streams = [None if m == lost else delta[m].reshape(-1) for m in range(M)]
        dh, _ = ne.ne_recover(streams, lost, p)
        assert torch.equal(dh.reshape(M, n, n).to(torch.int32), clean), lost
        del dh


def test_batch_256_sampled(ne, orc):
    """The batched workload (256 problems, sizes 64..2048): every
    convolution and permutation problem whole, and two rows of every GEMM
    problem, against the oracle."""
    recipe = ne_synth.batch_recipe(ne_synth.BASE_SEED + 3, 256, 64, 2048)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    probs = []
    for i, q in enumerate(recipe):
        r = i % q["M"]
        if q["op"] == 0:
            probs.append(ne.Problem(ne.NE_OP_GEMM, t(q["c"]), t(q["G"].T), r_check=r))
        elif q["op"] == 1:
            probs.append(ne.Problem(ne.NE_OP_CONV, t(q["c"]), t(q["g"]), r_check=r))
        else:
            probs.append(ne.Problem(ne.NE_OP_PERM, t(q["c"]), None, perm=t(q["perm"]),
                                    scale=t(q["scale"]), add=t(q["add"]), r_check=r))
    b = ne.Batch(probs)
    b.run()
    torch.cuda.synchronize()
    for i, (pb, q) in enumerate(zip(probs, recipe)):
        r = i % q["M"]
        assert int(pb.n_bad.item()) == 0, i
        got = pb.d_hat.cpu().numpy().astype(np.int64)
        if q["op"] == 0:
            s = q["c"].shape[1]
            for row in sorted({0, s - 1}):
                ref = orc.gemm_pipeline(q["c"][:, row:row + 1, :], q["G"], r=r)["dhat"][:, 0, :]
                want = ref.astype(np.int32).astype(np.int64) if pb.out_dtype == torch.int32 else ref
                assert np.array_equal(got[:, row, :], want), (i, row)
        elif q["op"] == 1:
            ref = orc.conv_pipeline(q["c"].astype(np.int64), q["g"].astype(np.int64), r=r)
            want = ref["dhat"]
            if pb.out_dtype == torch.int32:
                want = want.astype(np.int32).astype(np.int64)
            assert np.array_equal(got, want), i
        else:
            ref = orc.permute_scale_pipeline(q["c"].astype(np.int64), q["perm"], q["scale"],
                                             q["add"], r=r)
            want = ref["dhat"]
            if pb.out_dtype == torch.int32:
                want = want.astype(np.int32).astype(np.int64)
            assert np.array_equal(got, want), i
