"""The filter with room for k >= 2 block states runs block b on internal
stream b mod k (at most 4); every column must come out bit-identical to the
one-stream order (blocks are uncoupled and every kernel is deterministic),
also for a ragged last block, in FP64 and FP32."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("prec", [0, 1])
def test_two_stream_blocks_bit_identical(prec):
    from oracle import chfsi
    from oracle.paw import PAWOperator
    from paper_2604_26037_amd import Operator
    from workloads import make_system
    s = make_system("mid")
    ref = PAWOperator(s)
    op = Operator(s)
    N, B, m = 70, 16, 9                      # 5 blocks, the last one ragged (6 columns)
    X = torch.from_numpy(s.trial(N)).to("cuda:0")
    lam, _ = op.rayleigh_ritz(X)
    a = lam.cpu().numpy()
    bU = 1.02 * chfsi.lanczos_bounds(ref, k=25)[1] + 1.0
    one = op.workspace(op.cheb_filter_workspace(B, B, prec))
    two = op.workspace(op.cheb_filter_workspace(N, B, prec))
    assert two.numel() == 2 * one.numel()
    y1 = op.cheb_filter(X, lam, m, float(a[0]), float(a[-1]), bU, block=B, prec=prec, ws=one)
    y2 = op.cheb_filter(X, lam, m, float(a[0]), float(a[-1]), bU, block=B, prec=prec, ws=two)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(y1.cpu().numpy(), y2.cpu().numpy())
    three = op.workspace(3 * one.numel())
    y3 = op.cheb_filter(X, lam, m, float(a[0]), float(a[-1]), bU, block=B, prec=prec, ws=three)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(y1.cpu().numpy(), y3.cpu().numpy())
    if prec == 0:
        want = chfsi.rchfsi_filter(ref, X.cpu().numpy(), a, m, float(a[0]), float(a[-1]), bU, block=B)
        err = np.linalg.norm(y2.cpu().numpy() - want) / np.linalg.norm(want)
        assert err < 1e-9, err


def test_operators_share_block_streams():
    """Two operators (the mid workload and a graded GGA one) run two-stream
    filters on the library's shared block streams, interleaved on one caller
    stream, and on a second caller stream: each output equals that
    operator's one-stream result bit for bit, and an operator destroyed in
    between leaves the streams usable."""
    from paper_2604_26037_amd import Operator
    from workloads import make_system
    from workloads.configs import with_two_level_gga
    sa = make_system("mid")
    sb = with_two_level_gga(make_system("mid"), r_fine=1.0)
    N, B, m = 48, 16, 7
    runs = {}
    for name, s in (("a", sa), ("b", sb)):
        op = Operator(s)
        X = torch.from_numpy(s.trial(N)).to("cuda:0")
        lam, _ = op.rayleigh_ritz(X)
        a = lam.cpu().numpy()
        _, tmax, beta = op.lanczos_bounds(k=20)
        bU = 1.02 * (tmax + beta) + 1.0
        args = (lam, m, float(a[0]), float(a[-1]), bU)
        one = op.workspace(op.cheb_filter_workspace(B, B, 1))
        y1 = op.cheb_filter(X, *args, block=B, prec=1, ws=one)
        runs[name] = (op, X, args, y1.cpu().numpy())
    ws = {k: v[0].workspace(v[0].cheb_filter_workspace(N, B, 1)) for k, v in runs.items()}
    outs = {}
    for rep in range(2):
        for name in ("a", "b"):
            op, X, args, _ = runs[name]
            outs[(name, rep)] = op.cheb_filter(X, *args, block=B, prec=1, ws=ws[name])
    torch.cuda.synchronize()   # the side stream reuses operator b's workspace
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        op, X, args, _ = runs["b"]
        outs[("b", "side")] = op.cheb_filter(X, *args, block=B, prec=1, ws=ws["b"], stream=side)
    side.synchronize()
    torch.cuda.synchronize()
    for (name, _), y in outs.items():
        np.testing.assert_array_equal(y.cpu().numpy(), runs[name][3])
    # destroying one operator leaves the shared streams to the other
    del ws["a"], outs
    runs.pop("a")
    op, X, args, y_ref = runs["b"]
    y = op.cheb_filter(X, *args, block=B, prec=1, ws=ws["b"])
    torch.cuda.synchronize()
    np.testing.assert_array_equal(y.cpu().numpy(), y_ref)
