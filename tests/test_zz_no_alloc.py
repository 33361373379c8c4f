"""pam_eval_noalloc (the evaluation entry point that allocates nothing)
against pam_eval, through the C ABI: same kernels, so the values must agree
bit for bit, on two calls in a row (the second smaller, in the other query
precision, over two fields), with the out-of-domain counter; inputs beyond
the fixed scratch are refused before anything runs."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_2605_16564_amd import api, native, synth  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = api.Context(0)
    yield c
    c.close()


def test_noalloc_eval_matches_eval(ctx):
    g = synth.circle64()
    S = api.partition(ctx, g)
    D = api.init_lattice(ctx, g, [16, 16], 256)
    beta, _ = api.fit(ctx, S, D, api.EnetOpts(synth.LAMBDA1, synth.LAMBDA2, "f64"))
    # call 1: 600k FP32 queries, some outside the domain
    xq = torch.as_tensor(synth.uniform_queries(2, 600_000, seed=41, lo=[-0.05, 0.0],
                                               hi=[1.05, 1.0]), device="cuda")
    print("case noalloc call 1: circle64, 600k f32 queries", flush=True)
    n1 = torch.zeros(1, dtype=torch.int64, device="cuda")
    n2 = torch.zeros(1, dtype=torch.int64, device="cuda")
    ref = api.evaluate(ctx, g, D, beta, xq, n_outside=n1)
    got = torch.full_like(ref, 123.0)
    api.evaluate_noalloc(ctx, g, D, beta, xq, got, n_outside=n2)
    torch.cuda.synchronize()
    assert n1.item() == n2.item() and n1.item() > 0
    assert torch.equal(torch.isnan(ref), torch.isnan(got))
    fin = ~torch.isnan(ref)
    assert torch.equal(ref[fin], got[fin])
    # call 2: smaller, FP64 queries, two fields (the fit's subdomains twice)
    print("case noalloc call 2: two fields, 5k f64 queries", flush=True)
    D2 = api.concat_dicts([D, D])
    b2 = torch.cat([beta, beta])
    xq2 = torch.as_tensor(synth.uniform_queries(2, 5_000, seed=42, dtype=np.float64), device="cuda")
    ref2 = api.evaluate(ctx, [g, g], D2, b2, xq2, q_counts=[2_000, 3_000], space=1)
    got2 = torch.empty_like(ref2)
    api.evaluate_noalloc(ctx, [g, g], D2, b2, xq2, got2, q_counts=[2_000, 3_000], space=1)
    torch.cuda.synchronize()
    assert torch.equal(ref2, got2)


def test_noalloc_limits(ctx):
    g = synth.circle64()
    D = api.init_lattice(ctx, g, [16, 16], 256)
    beta = torch.zeros((4, 256), dtype=torch.float64, device="cuda")
    Q = 6_000_000                      # about 72 MB of binning workspace > 64 MiB
    xq = torch.zeros((Q, 2), dtype=torch.float32, device="cuda")
    out = torch.full((Q,), 5.0, dtype=torch.float32, device="cuda")
    with pytest.raises(native.PamError, match="64 MiB"):
        api.evaluate_noalloc(ctx, g, D, beta, xq, out)
    torch.cuda.synchronize()
    assert torch.all(out == 5.0)       # nothing ran
    with pytest.raises(native.PamError, match="8 fields"):
        api.evaluate_noalloc(ctx, [g] * 9, api.concat_dicts([D] * 9), beta.repeat(9, 1), xq[:90],
                             out[:90], q_counts=[10] * 9)
