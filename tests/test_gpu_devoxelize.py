"""De-voxelisation on the GPU against the FP64 oracle: max (and its argmax
slots) bit-exact - a max of float32 values is exact - and mean within float32
rounding; the backward of both reductions against the oracle's; slot indices
out of range are ignored, as documented."""

import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2512_20927_amd import _lib
    return _lib


def _case(seed, G=3000, U=2000, C=36, max_slots=12):
    rng = np.random.default_rng(seed)
    counts = rng.integers(0, max_slots + 1, G)
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    vu = rng.integers(0, U, offs[-1]).astype(np.int32)
    pred = rng.standard_normal((U, C)).astype(np.float32)
    pred[::7, ::5] = 0.25  # repeated values: ties resolved to the first slot
    return offs, vu, pred


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("reduce", ["max", "mean"])
def test_forward_and_backward_match_oracle(L, reduce):
    code = L.QR_REDUCE_MAX if reduce == "max" else L.QR_REDUCE_MEAN
    offs, vu, pred = _case(1)
    G, U, C = offs.size - 1, pred.shape[0], pred.shape[1]
    out = torch.full((G, C), float("nan"), device="cuda")
    arg = torch.full((G, C), -7, dtype=torch.int32, device="cuda") if reduce == "max" else None
    L.qr_devoxelize(_t(offs), _t(vu), _t(pred), code, out, arg)
    torch.cuda.synchronize()
    want, want_arg = oracle.devoxelize(offs, vu, pred.astype(np.float64), reduce)
    got = out.cpu().numpy()
    if reduce == "max":
        np.testing.assert_array_equal(got, want.astype(np.float32))
        np.testing.assert_array_equal(arg.cpu().numpy(), want_arg)
    else:
        np.testing.assert_allclose(got, want, rtol=2e-6, atol=2e-7)
    gout = np.random.default_rng(2).standard_normal((G, C)).astype(np.float32)
    grad = torch.zeros(U, C, device="cuda")
    L.qr_devoxelize_backward(_t(offs), _t(vu), U, code, _t(gout), arg, grad)
    torch.cuda.synchronize()
    want_g = oracle.devoxelize_backward(offs, vu, U, gout.astype(np.float64), reduce, want_arg)
    np.testing.assert_allclose(grad.cpu().numpy(), want_g, rtol=1e-5, atol=1e-6)


def test_out_of_range_slots_are_ignored(L):
    offs = np.array([0, 3, 3, 5], np.int64)
    vu = np.array([1, 99, 0, -4, 2], np.int32)  # 99 and -4 are outside [0, 3)
    pred = np.arange(12, dtype=np.float32).reshape(3, 4)
    out = torch.empty(3, 4, device="cuda")
    arg = torch.empty(3, 4, dtype=torch.int32, device="cuda")
    L.qr_devoxelize(_t(offs), _t(vu), _t(pred), L.QR_REDUCE_MAX, out, arg)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), [pred[1], np.zeros(4), pred[2]])
    np.testing.assert_array_equal(arg.cpu().numpy(), [[0] * 4, [-1] * 4, [4] * 4])
