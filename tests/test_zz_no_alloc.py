"""GPU checks of the allocation-free entry point ltl_run_noalloc, called through the C ABI:
its grid equals that of ltl_create + ltl_step + ltl_read (itself pinned to the oracle by the
parity tests) on two calls in a row, the second with a smaller grid (and another radius, so
the band table in the static device array is rewritten), plus the oracle on small cases."""
import numpy as np
import pytest
import torch

import oracle
from paper_2406_17284_amd import inputs, ltl

pytestmark = pytest.mark.gpu


def _handle_run(g0, rule, method, n, boundary):
    """The existing entry points: create, set boundary, step, read, destroy."""
    H, W = g0.shape
    pitch = ltl.ltl_pitch(W)
    nbytes = ltl.ltl_buffer_bytes(H, W, rule.R, method)
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    init = torch.from_numpy(g0).cuda()
    out = torch.empty((H, W), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    h = ltl.ltl_create(H, W, rule, method, a.data_ptr(), b.data_ptr(), nbytes, init.data_ptr(), W, 0)
    try:
        ltl.ltl_set_boundary(h, boundary)
        ltl.ltl_step(h, n)
        ltl.ltl_read(h, out.data_ptr(), W)
        torch.cuda.synchronize()
    finally:
        ltl.ltl_destroy(h)
    assert pitch >= W
    return out.cpu().numpy()


def _noalloc_run(g0, rule, method, n, boundary, bufs=None):
    H, W = g0.shape
    nbytes = ltl.ltl_buffer_bytes(H, W, rule.R, method)
    if bufs is None:
        bufs = (torch.empty(nbytes, dtype=torch.uint8, device="cuda"),
                torch.empty(nbytes, dtype=torch.uint8, device="cuda"))
    a, b = bufs
    assert a.numel() >= nbytes and b.numel() >= nbytes
    # stale contents must not matter: the call initializes both buffers itself
    a.fill_(7)
    b.fill_(9)
    init = torch.from_numpy(g0).cuda()
    out = torch.full((H, W), 5, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    ltl.ltl_run_noalloc(H, W, rule, method, boundary, a.data_ptr(), b.data_ptr(), a.numel(), init.data_ptr(), W, n,
                        out.data_ptr(), W, 0)
    torch.cuda.synchronize()
    pitch = ltl.ltl_pitch(W)
    # the padding columns of both buffers are dead after the run
    for buf in (a, b):
        pad = buf[: H * pitch].view(H, pitch)[:, W:]
        if pad.numel():
            assert int(pad.max().item()) == 0
    return out.cpu().numpy()


CASES = [
    # (first grid, rule, method, steps, boundary), then a smaller second call
    ("cat_i8", inputs.BOSCO_M1, (300, 420), (97, 130), inputs.Rule(2, 0, 1, 6, 11, 6, 8), 13, "dead"),
    ("cat_i8", inputs.Rule(16, 0, 1, 272, 490, 294, 370), (256, 320), (64, 96), inputs.LIFE, 9, "dead"),
    ("cat_f16", inputs.Rule(7, 0, 1, 56, 101, 60, 76), (200, 256), (80, 64), inputs.BOSCO_M1, 7, "periodic"),
    ("cat_f8", inputs.Rule(3, 0, 1, 12, 22, 13, 16), (160, 224), (48, 80), inputs.Rule(1, 0, 0, 2, 3, 3, 3), 11, "dead"),
    ("cat_i8", inputs.Rule(16, 8, 0, 300, 500, 330, 420), (192, 256), (64, 128), inputs.Rule(5, 4, 1, 34, 58, 34, 45),
     6, "dead"),
    ("direct", inputs.BOSCO_M1, (150, 200), (40, 33), inputs.LIFE, 5, "dead"),
]


@pytest.mark.parametrize("method,rule1,shape1,shape2,rule2,n,boundary", CASES)
def test_noalloc_matches_handle_on_two_calls(method, rule1, shape1, shape2, rule2, n, boundary):
    m = ltl.METHODS[method]
    bd = ltl.BOUNDARIES[boundary]
    p = 0.5 if rule1.C <= 2 else 0.42
    g1 = inputs.bernoulli_grid(*shape1, p, seed=11)
    g2 = inputs.bernoulli_grid(*shape2, 0.5, seed=12)
    # one pair of buffers for both calls, sized for the first (larger) grid
    nb = ltl.ltl_buffer_bytes(*shape1, max(rule1.R, rule2.R), m)
    bufs = (torch.empty(nb, dtype=torch.uint8, device="cuda"), torch.empty(nb, dtype=torch.uint8, device="cuda"))
    print(f"noalloc {method} {shape1} R{rule1.R} then {shape2} R{rule2.R}, {n} steps, {boundary}", flush=True)
    got1 = _noalloc_run(g1, rule1, m, n, bd, bufs)
    got2 = _noalloc_run(g2, rule2, m, n, bd, bufs)
    ref1 = _handle_run(g1, rule1, m, n, bd)
    ref2 = _handle_run(g2, rule2, m, n, bd)
    assert np.array_equal(got1, ref1), f"first call differs in {(got1 != ref1).sum()} cells"
    assert np.array_equal(got2, ref2), f"second call differs in {(got2 != ref2).sum()} cells"
    if shape2[0] * shape2[1] <= 64 * 128:
        ref_o = oracle.run(g2, rule2, n, periodic=(boundary == "periodic"))
        assert np.array_equal(got2, ref_o)


def test_noalloc_zero_steps_and_refusals():
    g = inputs.bernoulli_grid(40, 50, 0.5, seed=3)
    got = _noalloc_run(g, inputs.LIFE, ltl.LTL_CAT_I8, 0, ltl.LTL_BOUNDARY_DEAD)
    assert np.array_equal(got, g)
    nb = ltl.ltl_buffer_bytes(40, 50, 1, ltl.LTL_CAT_I8)
    a = torch.empty(nb, dtype=torch.uint8, device="cuda")
    b = torch.empty(nb, dtype=torch.uint8, device="cuda")
    init = torch.from_numpy(g).cuda()
    out = torch.empty((40, 50), dtype=torch.uint8, device="cuda")
    with pytest.raises(ltl.LtlError) as e:   # buffers too small
        ltl.ltl_run_noalloc(40, 50, inputs.LIFE, ltl.LTL_CAT_I8, 0, a.data_ptr(), b.data_ptr(), nb - 1,
                            init.data_ptr(), 50, 3, out.data_ptr(), 50, 0)
    assert e.value.code == ltl.LTL_ERR_SIZE
    with pytest.raises(ltl.LtlError) as e:   # periodic needs W % 16 == 0
        ltl.ltl_run_noalloc(40, 50, inputs.LIFE, ltl.LTL_CAT_I8, 1, a.data_ptr(), b.data_ptr(), nb,
                            init.data_ptr(), 50, 3, out.data_ptr(), 50, 0)
    assert e.value.code == ltl.LTL_ERR_UNSUPPORTED


def test_noalloc_on_a_side_stream():
    g = inputs.bernoulli_grid(128, 192, 0.5, seed=5)
    rule = inputs.BOSCO_M1
    nb = ltl.ltl_buffer_bytes(128, 192, rule.R, ltl.LTL_CAT_I8)
    a = torch.empty(nb, dtype=torch.uint8, device="cuda")
    b = torch.empty(nb, dtype=torch.uint8, device="cuda")
    init = torch.from_numpy(g).cuda()
    out = torch.empty((128, 192), dtype=torch.uint8, device="cuda")
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    ltl.ltl_run_noalloc(128, 192, rule, ltl.LTL_CAT_I8, 0, a.data_ptr(), b.data_ptr(), nb, init.data_ptr(), 192, 10,
                        out.data_ptr(), 192, side)
    side.synchronize()
    assert np.array_equal(out.cpu().numpy(), oracle.run(g, rule, 10))
