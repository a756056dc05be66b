"""bench.py's host-side contract, checked without a GPU: more than one GPU
is refused with a message and exit status 2 before anything touches a
device, and every workload the help lists is one the script dispatches."""

import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_every_listed_workload_is_dispatched():
    src = open(os.path.join(ROOT, "bench.py")).read()
    listed = re.search(r'"--workload", default="room", choices=\[([^\]]*)\]', src).group(1)
    names = re.findall(r'"(\w+)"', listed)
    assert {"room", "rgb", "devox", "batched", "diff", "precision"} <= set(names)
    for n in names:
        assert re.search(r'"%s": run_%s\b' % (n, n), src), n


def test_oracle_tile_equals_the_full_frame_render():
    """bench.oracle_tile renders one tile as its own image with the records
    shifted by the tile origin; that must be exactly the full-frame render of
    the tile (ragged edge tiles included)."""
    import numpy as np
    import bench
    import oracle
    import synth
    sc, cam = synth.make_tiny(3, n=800, dim=16), synth.tiny_camera(40)
    cam.height, cam.cy = 37, 18.5
    pr = oracle.project(sc.means, sc.scales, sc.quats, sc.opacity, cam)
    tx, ty = 3, 3
    gids, offs, _ = oracle.bin_sort(pr["rect"], pr["depth"], tx, ty)
    rec = dict(means2d=pr["means2d"], conic=pr["conic"], opacity=pr["opacity"], gids=gids, offs=offs)
    full_q = oracle.render_quantile(pr, gids, offs, sc.features, 40, 37, 8)
    full_d = oracle.render_dense(pr, gids, offs, sc.features, 40, 37)
    for t in range(tx * ty):
        y0, x0 = (t // tx) * 16, (t % tx) * 16
        q = bench.oracle_tile(rec, t, sc.features, 40, 37, 8)
        d = bench.oracle_tile(rec, t, sc.features, 40, 37)
        h, w = q["out"].shape[:2]
        assert (h, w) == (min(16, 37 - y0), min(16, 40 - x0))
        np.testing.assert_array_equal(q["out"], full_q["out"][y0:y0 + h, x0:x0 + w])
        np.testing.assert_array_equal(q["margin"], full_q["margin"][y0:y0 + h, x0:x0 + w])
        np.testing.assert_array_equal(d["out"], full_d["out"][y0:y0 + h, x0:x0 + w])


def test_counter_summary_blocks_and_source_hash(tmp_path, monkeypatch):
    """A summary file of several kernels: each kernel's traffic comes from
    its own block, and a block whose source hash no longer matches the
    sources gives no traffic."""
    import bench
    from paper_2512_20927_amd import profile_summary as ps
    cur = ps.source_hash("quantile_backward")
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "two_pmc.txt").write_text(
        "# header: ignored\n\n"
        "kernel: first_kernel\ntraffic_bytes_per_launch: 111\nsource_sha256: %s\n\n"
        "kernel: second_kernel\ntraffic_bytes_per_launch: 222\nsource_sha256: %s\n" % (cur, "0" * 16))
    got = ps.read_summary(str(tmp_path / "profiles" / "two_pmc.txt"), kernel="first_kernel")
    assert got["traffic_bytes_per_launch"] == "111" and got["source_sha256"] == cur
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("first_kernel<1>", "x", "quantile_backward", summary="two_pmc.txt") == 111
    assert bench.measured_traffic("second_kernel", "x", "quantile_backward", summary="two_pmc.txt") is None
    assert bench.measured_traffic("third_kernel", "x", "quantile_backward", summary="two_pmc.txt") is None
