"""The C-ABI library loads on a machine without a GPU, exports every entry
point include/qrender.h declares, and rejects bad arguments on the host
before any HIP call (no compute call is made here)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qrender.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qr_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_2512_20927_amd import _lib
    return _lib


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert len(names) >= 11
    for n in names:
        assert hasattr(L.lib(), n), n
    assert sorted(L.EXPORTED) == names


def test_version(L):
    assert L.version().startswith("qrender")


def _err(L, rc):
    return rc, L.last_error()


def test_project_validation(L):
    lib = L.lib()
    cam = L.make_camera(type("C", (), dict(R_cw=[1, 0, 0, 0, 1, 0, 0, 0, 1], t=[0, 0, 3], fx=50.0,
                                             fy=50.0, cx=32.0, cy=32.0, width=64, height=64,
                                             z_near=0.2))())
    prm = L.make_params()
    nul = None
    rc, msg = _err(L, lib.qr_project(nul, -1, nul, nul, nul, nul, ctypes.byref(cam), ctypes.byref(prm), nul, nul, nul, nul, nul))
    assert rc == L.QR_ERR_INVALID_ARG and "n < 0" in msg
    rc, msg = _err(L, lib.qr_project(nul, 10, nul, nul, nul, nul, ctypes.byref(cam), ctypes.byref(prm), nul, nul, nul, nul, nul))
    assert rc == L.QR_ERR_INVALID_ARG and "null" in msg
    rc, _ = _err(L, lib.qr_project(nul, 10, nul, nul, nul, nul, None, ctypes.byref(prm), nul, nul, nul, nul, nul))
    assert rc == L.QR_ERR_INVALID_ARG
    bad = L.make_camera(type("C", (), dict(R_cw=[1, 0, 0, 0, 1, 0, 0, 0, 1], t=[0, 0, 3], fx=-1.0,
                                             fy=50.0, cx=32.0, cy=32.0, width=64, height=64))())
    rc, msg = _err(L, lib.qr_project(nul, 10, nul, nul, nul, nul, ctypes.byref(bad), ctypes.byref(prm), nul, nul, nul, nul, nul))
    assert rc == L.QR_ERR_INVALID_ARG and "focal" in msg
    badp = L.make_params(alpha_min=0.0)
    rc, _ = _err(L, lib.qr_project(nul, 10, nul, nul, nul, nul, ctypes.byref(cam), ctypes.byref(badp), nul, nul, nul, nul, nul))
    assert rc == L.QR_ERR_INVALID_ARG
    # n = 0 is a valid no-op
    assert lib.qr_project(nul, 0, nul, nul, nul, nul, ctypes.byref(cam), ctypes.byref(prm), nul, nul, nul, nul, nul) == L.QR_OK


def test_bin_sort_validation_and_workspace_size(L):
    lib = L.lib()
    out = ctypes.c_size_t(0)
    assert lib.qr_bin_sort_workspace_size(1000, 4, 4, 5000, ctypes.byref(out)) == L.QR_OK
    small = out.value
    assert lib.qr_bin_sort_workspace_size(1000, 4, 4, 50000, ctypes.byref(out)) == L.QR_OK
    assert out.value > small > 5000 * 16
    assert lib.qr_bin_sort_workspace_size(-1, 4, 4, 10, ctypes.byref(out)) == L.QR_ERR_INVALID_ARG
    assert lib.qr_bin_sort_workspace_size(10, 0, 4, 10, ctypes.byref(out)) == L.QR_ERR_INVALID_ARG
    dummy = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    rc = lib.qr_bin_sort(None, 1000, 4, 4, dummy, dummy, dummy, 5000, dummy, 16, dummy, None, dummy, dummy)
    assert rc == L.QR_ERR_CAPACITY and "workspace" in L.last_error()
    rc = lib.qr_bin_sort(None, 1000, 4, 4, None, dummy, dummy, 5000, dummy, 1 << 30, dummy, None, dummy, dummy)
    assert rc == L.QR_ERR_INVALID_ARG
    rc = lib.qr_bin_sort(None, 1 << 33, 4, 4, dummy, dummy, dummy, 5000, dummy, 1 << 30, dummy, None, dummy, dummy)
    assert rc == L.QR_ERR_UNSUPPORTED


def test_bin_sort_noalloc_rejects_sizes_beyond_its_scratch(L):
    """The static-workspace binning refuses, before touching a device, any
    size whose workspace would not fit its fixed scratch array."""
    lib = L.lib()
    dummy = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    out = ctypes.c_size_t(0)
    cap = 4_300_000
    assert lib.qr_bin_sort_workspace_size(1000, 40, 30, cap, ctypes.byref(out)) == L.QR_OK
    assert out.value > L.QR_BIN_SORT_SCRATCH_BYTES
    rc = lib.qr_bin_sort_noalloc(None, 1000, 40, 30, dummy, dummy, dummy, cap, dummy, None, dummy, dummy)
    assert rc == L.QR_ERR_CAPACITY and "scratch" in L.last_error()
    rc = lib.qr_bin_sort_noalloc(None, 1000, 40, 30, dummy, dummy, dummy, 1 << 40, dummy, None, dummy, dummy)
    assert rc == L.QR_ERR_CAPACITY
    rc = lib.qr_bin_sort_noalloc(None, 1000, 0, 30, dummy, dummy, dummy, 100, dummy, None, dummy, dummy)
    assert rc == L.QR_ERR_INVALID_ARG


def test_render_validation(L):
    lib = L.lib()
    prm = L.make_params()
    d = ctypes.c_void_p(0x1000)
    P = ctypes.byref(prm)
    q = lambda W, H, K, dt, sc, dim, sg=None, sw=None, tf=None, lp=None, prm=P: lib.qr_render_quantile(
        None, W, H, prm, K, d, d, d, d, d, dt, sc, dim, d, None, None, tf, lp, sg, sw)
    assert q(0, 64, 8, 0, None, 16) == L.QR_ERR_INVALID_ARG
    assert q(64, 64, 0, 0, None, 16) == L.QR_ERR_UNSUPPORTED
    assert q(64, 64, L.QR_MAX_K + 1, 0, None, 16) == L.QR_ERR_UNSUPPORTED
    # T_final / last_pos are Algorithm 1's outputs only
    strat_p = ctypes.byref(L.make_params(selection=L.QR_SELECT_STRATIFIED))
    assert q(64, 64, 8, 0, None, 16, tf=d, prm=strat_p) == L.QR_ERR_UNSUPPORTED
    assert q(64, 64, 8, 0, None, 16, lp=d, prm=strat_p) == L.QR_ERR_UNSUPPORTED
    assert q(64, 64, 8, 0, None, 24) == L.QR_ERR_UNSUPPORTED
    assert q(64, 64, 8, 0, None, 0) == L.QR_ERR_UNSUPPORTED
    assert q(64, 64, 8, 7, None, 16) == L.QR_ERR_UNSUPPORTED
    assert q(64, 64, 8, 2, None, 16) == L.QR_ERR_INVALID_ARG  # fp8 without scale
    assert q(64, 64, 8, 0, None, 16, sg=d) == L.QR_ERR_INVALID_ARG  # sel_gid without sel_w
    rc = lib.qr_render_dense(None, 64, 64, P, d, d, d, d, None, 0, None, 16, d, None, None)
    assert rc == L.QR_ERR_INVALID_ARG
    rc = lib.qr_render_dense(None, 64, 64, None, d, d, d, d, d, 0, None, 16, d, None, None)
    assert rc == L.QR_ERR_INVALID_ARG
    rc = lib.qr_render_dense_backward(None, 64, 64, P, d, d, d, d, d, 0, None, 20, d, d, d, d, d)
    assert rc == L.QR_ERR_UNSUPPORTED
    rc = lib.qr_render_quantile_backward(None, 64, 64, P, L.QR_MAX_K + 1, d, d, d, d, d, 0, None, 16, d,
                                         d, d, d)
    assert rc == L.QR_ERR_UNSUPPORTED
    # output dtype: bf16 maps from Q-Render only; unknown codes rejected
    bad_out = L.make_params(out_dtype=7)
    rc = lib.qr_render_quantile(None, 64, 64, ctypes.byref(bad_out), 8, d, d, d, d, d, 0, None, 16, d,
                                None, None, None, None, None, None)
    assert rc == L.QR_ERR_UNSUPPORTED and "output dtype" in L.last_error()
    bf_out = L.make_params(out_dtype=L.QR_BF16)
    rc = lib.qr_render_dense(None, 64, 64, ctypes.byref(bf_out), d, d, d, d, d, 0, None, 16, d, None, None)
    assert rc == L.QR_ERR_UNSUPPORTED and "float32 output" in L.last_error()
    rc = lib.qr_render_quantile_batched(None, 1, d, ctypes.byref(bad_out), 8, 0, 16, d, 10, 0, None, 0)
    assert rc == L.QR_ERR_UNSUPPORTED
    bad_sel = L.make_params(selection=5)
    rc = lib.qr_render_quantile(None, 64, 64, ctypes.byref(bad_sel), 8, d, d, d, d, d, 0, None, 16, d,
                                None, None, None, None, None, None)
    assert rc == L.QR_ERR_UNSUPPORTED and "selection" in L.last_error()
    rc = lib.qr_render_quantile_batched(None, 1, d, ctypes.byref(bad_sel), 8, 0, 16, d, 10, 0, None, 0)
    assert rc == L.QR_ERR_UNSUPPORTED
    strat = L.make_params(selection=L.QR_SELECT_STRATIFIED)
    rc = lib.qr_render_quantile_backward(None, 64, 64, ctypes.byref(strat), 8, d, d, d, d, d, 0, None,
                                         16, d, d, d, d)
    assert rc == L.QR_ERR_UNSUPPORTED
    rc = lib.qr_quantize_features(None, 10, 16, d, 0, d, None)
    assert rc == L.QR_ERR_UNSUPPORTED
    rc = lib.qr_quantize_features(None, 10, 16, d, 2, d, None)
    assert rc == L.QR_ERR_INVALID_ARG


def test_batched_validation(L):
    lib = L.lib()
    prm = L.make_params()
    P = ctypes.byref(prm)
    d = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first

    def b(n_views, n_items, n_wg, ws, ws_bytes, K=8, dtype=0, dim=16):
        return lib.qr_render_quantile_batched(None, n_views, d, P, K, dtype, dim, d, n_items,
                                              n_wg, ws, ws_bytes)

    assert b(0, 10, 0, None, 0) == L.QR_ERR_INVALID_ARG
    assert b(1, 10, -1, None, 0) == L.QR_ERR_INVALID_ARG
    assert b(1, 10, 4, None, 0) == L.QR_ERR_CAPACITY  # persistent mode needs the counter
    assert b(1, 10, 4, d, 2) == L.QR_ERR_CAPACITY
    assert b(1, 10, 4, d, 16) == L.QR_ERR_CAPACITY  # one 4-byte counter per XCD
    assert b(1, 1 << 31, 0, None, 0) == L.QR_ERR_INVALID_ARG
    assert b(1, 10, 0, None, 0, K=0) == L.QR_ERR_UNSUPPORTED
    assert b(1, 10, 0, None, 0, dtype=9) == L.QR_ERR_UNSUPPORTED
    assert b(1, 10, 0, None, 0, dim=24) == L.QR_ERR_UNSUPPORTED
    assert b(1, 0, 0, None, 0) == L.QR_OK  # nothing to render: no launch
    def bb(n_views, n_items, n_wg, ws, ws_bytes, K=8, dtype=0, dim=16, grads=d):
        return lib.qr_render_quantile_batched_backward(None, n_views, d, grads, P, K, dtype, dim, d,
                                                       n_items, n_wg, ws, ws_bytes)

    assert bb(0, 10, 0, None, 0) == L.QR_ERR_INVALID_ARG
    assert bb(1, 10, 0, None, 0, grads=None) == L.QR_ERR_INVALID_ARG
    assert bb(1, 10, -1, None, 0) == L.QR_ERR_INVALID_ARG
    assert bb(1, 10, 4, d, 16) == L.QR_ERR_CAPACITY
    assert bb(1, 1 << 31, 0, None, 0) == L.QR_ERR_INVALID_ARG
    assert bb(1, 10, 0, None, 0, K=L.QR_MAX_K + 1) == L.QR_ERR_UNSUPPORTED
    assert bb(1, 10, 0, None, 0, dtype=9) == L.QR_ERR_UNSUPPORTED
    assert bb(1, 10, 0, None, 0, dim=24) == L.QR_ERR_UNSUPPORTED
    assert bb(1, 0, 0, None, 0) == L.QR_OK
    rc = lib.qr_batch_schedule(None, 0, d, d, 10, d, d, 256)
    assert rc == L.QR_ERR_INVALID_ARG
    # autotuner: host-side argument checks before any launch
    sch = (ctypes.c_void_p * 2)(0x1000, 0x1000)
    wg = (ctypes.c_int32 * 2)(0, 3)
    times = (ctypes.c_float * 4)()
    bi, bw = ctypes.c_int32(), ctypes.c_int32()

    def at(n_sched=2, n_wg=2, reps=2, schedules=sch, wgs=wg, t=times):
        return lib.qr_autotune_batched(None, 1, d, P, 8, 0, 16, schedules, n_sched, 10, wgs, n_wg, reps,
                                       d, 64, t, ctypes.byref(bi), ctypes.byref(bw))

    assert at(reps=0) == L.QR_ERR_INVALID_ARG
    assert at(n_sched=0) == L.QR_ERR_INVALID_ARG
    assert at(t=None) == L.QR_ERR_INVALID_ARG
    assert at(schedules=(ctypes.c_void_p * 2)(0x1000, None)) == L.QR_ERR_INVALID_ARG
    assert at(wgs=(ctypes.c_int32 * 2)(0, 65)) == L.QR_ERR_INVALID_ARG
    rc = lib.qr_batch_schedule(None, 2, d, d, 10, d, d, 16)
    assert rc == L.QR_ERR_CAPACITY


def test_devoxelize_validation(L):
    lib = L.lib()
    d = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    dv = lambda G, C, red, offs=d, vu=d, M=10, out=d: lib.qr_devoxelize(None, G, C, offs, vu, M, 5, d, red, out, None)
    assert dv(-1, 16, 0) == L.QR_ERR_INVALID_ARG
    assert dv(10, 6, 0) == L.QR_ERR_UNSUPPORTED  # dim not a multiple of 4
    assert dv(10, 16, 3) == L.QR_ERR_UNSUPPORTED
    assert dv(10, 16, 0, offs=None) == L.QR_ERR_INVALID_ARG
    assert dv(10, 16, 0, out=None) == L.QR_ERR_INVALID_ARG
    assert dv(0, 16, 0) == L.QR_OK  # nothing to do
    rc = lib.qr_devoxelize_backward(None, 10, 16, d, d, 10, 5, 0, d, None, d)
    assert rc == L.QR_ERR_INVALID_ARG  # max needs the argmax slots



def test_sh_to_rgb_validation(L):
    lib = L.lib()
    d = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    cam = L.make_camera(type("C", (), dict(R_cw=[1, 0, 0, 0, 1, 0, 0, 0, 1], t=[0, 0, 3], fx=50.0,
                                           fy=50.0, cx=32.0, cy=32.0, width=64, height=64))())
    cp = ctypes.byref(cam)
    sh = lambda n=10, deg=3, stride=16, c=cp, out_dim=16, m=d: lib.qr_sh_to_rgb(None, n, deg, m, d, stride, c, d,
                                                                                 out_dim)
    assert sh(n=-1) == L.QR_ERR_INVALID_ARG
    assert sh(deg=4) == L.QR_ERR_UNSUPPORTED
    assert sh(deg=-1) == L.QR_ERR_UNSUPPORTED
    assert sh(stride=15) == L.QR_ERR_INVALID_ARG  # degree 3 needs 16 coefficients
    assert sh(out_dim=2) == L.QR_ERR_INVALID_ARG
    assert sh(c=None) == L.QR_ERR_INVALID_ARG
    assert sh(m=None) == L.QR_ERR_INVALID_ARG
    assert sh(n=0) == L.QR_OK  # nothing to do
    cams = L.make_cameras([cam, cam])
    shv = lambda n=10, nv=2, c=cams: lib.qr_sh_to_rgb_views(None, n, 3, d, d, 16, c, nv, d, 16)
    assert shv(nv=0) == L.QR_ERR_INVALID_ARG
    assert shv(c=None) == L.QR_ERR_INVALID_ARG
    assert shv(n=-1) == L.QR_ERR_INVALID_ARG
    assert lib.qr_sh_to_rgb_views(None, 10, 5, d, d, 16, cams, 2, d, 16) == L.QR_ERR_UNSUPPORTED
    assert lib.qr_sh_to_rgb_views(None, 10, 3, d, d, 16, cams, 2, d, 6) == L.QR_ERR_UNSUPPORTED
    assert shv(n=0) == L.QR_OK

def test_views_front_validation(L):
    lib = L.lib()
    prm = L.make_params()
    d = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    mk = lambda **kw: dict(dict(R_cw=[1, 0, 0, 0, 1, 0, 0, 0, 1], t=[0, 0, 3], fx=50.0, fy=50.0,
                                cx=32.0, cy=32.0, width=64, height=64, z_near=0.2), **kw)
    cams = L.make_cameras([type("C", (), mk())(), type("C", (), mk(t=[0, 0, 4]))()])
    pv = lambda n, nv, cs: lib.qr_project_views(None, n, d, d, d, d, nv, cs, ctypes.byref(prm),
                                                d, d, d, d, d)
    assert pv(10, 0, cams) == L.QR_ERR_INVALID_ARG
    assert pv(-1, 2, cams) == L.QR_ERR_INVALID_ARG
    other = L.make_cameras([type("C", (), mk())(), type("C", (), mk(width=80))()])
    rc = pv(10, 2, other)
    assert rc == L.QR_ERR_INVALID_ARG and "image size" in L.last_error()
    bad = L.make_cameras([type("C", (), mk())(), type("C", (), mk(fx=0.0))()])
    assert pv(10, 2, bad) == L.QR_ERR_INVALID_ARG
    assert pv(0, 2, cams) == L.QR_OK  # no Gaussians: nothing to launch
    rc = lib.qr_project_views(None, 10, None, d, d, d, 2, cams, ctypes.byref(prm), d, d, d, d, d)
    assert rc == L.QR_ERR_INVALID_ARG
    bs = lambda nv, npv, ws_bytes: lib.qr_bin_sort_views(None, nv, npv, 4, 4, d, d, d, 5000, d,
                                                         ws_bytes, d, None, d, d)
    assert bs(0, 100, 1 << 30) == L.QR_ERR_INVALID_ARG
    assert bs(2, -1, 1 << 30) == L.QR_ERR_INVALID_ARG
    out = ctypes.c_size_t(0)
    assert lib.qr_bin_sort_workspace_size(3 * 100, 4, 3 * 4, 5000, ctypes.byref(out)) == L.QR_OK
    assert bs(3, 100, out.value - 1) == L.QR_ERR_CAPACITY
    assert bs(2, 1 << 32, 1 << 30) == L.QR_ERR_UNSUPPORTED


def test_count_pairs_validation(L):
    lib = L.lib()
    out = ctypes.c_uint64(7)
    assert lib.qr_count_pairs(None, 0, None, None, 0, ctypes.byref(out)) == L.QR_OK and out.value == 0
    d = ctypes.c_void_p(0x1000)
    assert lib.qr_count_pairs(None, 5, d, d, 4, ctypes.byref(out)) == L.QR_ERR_CAPACITY
    assert lib.qr_count_pairs(None, 5, None, d, 8, ctypes.byref(out)) == L.QR_ERR_INVALID_ARG


def test_product_path_does_not_touch_the_oracle():
    """The package sources never import, load or run anything under oracle/."""
    pkg = os.path.join(ROOT, "paper_2512_20927_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"\boracle\b", src), f


def test_binding_constants_match_the_header(L):
    """Every enumerator and #define constant the binding mirrors has the
    header's value (the selection rules, reductions, dtypes, error codes,
    limits)."""
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    values = {m.group(1): int(m.group(2)) for m in re.finditer(r"\b(QR_[A-Z0-9_]+)\s*=\s*(-?\d+)", src)}
    values.update({m.group(1): int(m.group(2)) for m in re.finditer(r"#define\s+(QR_[A-Z0-9_]+)\s+(\d+)\b", src)})
    mirrored = [n for n in dir(L) if n.startswith("QR_") and isinstance(getattr(L, n), int)]
    assert {"QR_SELECT_TOPK", "QR_SELECT_STRATIFIED", "QR_REDUCE_MEAN", "QR_FP8_E4M3"} <= set(mirrored)
    for n in mirrored:
        assert n in values, n
        assert getattr(L, n) == values[n], (n, getattr(L, n), values[n])
