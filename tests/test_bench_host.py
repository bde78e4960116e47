"""Host logic of bench.py: the algorithmic per-cell figures its roofline divides
by, pinned to the oracle's stencil definitions (section 3.1: S0 = {|i|^2 <= R^2},
the ball of radius R - 1 and the 2d biased cones; section 3.3: the derivative
rows of the smoothness indicators; section 5.1: the face Gauss points), and
the readers of the committed counter summaries, which must give nothing once
the kernel sources differ from those the summary was taken with."""
import os
import shutil

import pytest

import bench
from oracle import weights as ow


@pytest.mark.parametrize("d,R", [(2, 2), (2, 3), (3, 2), (3, 3)])
def test_stencil_shapes_match_the_oracle(d, R):
    sn, npts, nder, nst, n0 = bench._SHAPES[(d, R)]
    subs = ow.substencils(d, R)
    assert n0 == len(ow.full_stencil(d, R))
    assert nst == len(subs)
    assert sn == sum(len(s) for s in subs)
    assert npts == len(ow.face_points(d, R))
    assert nder == len(ow.derivative_indices(d, R))


def test_per_cell_figures():
    # three float64 averages per variable and cell: stage input, step start, new value
    assert bench.state_bytes_per_cell(3) == 3 * 8 * 5
    assert bench.state_bytes_per_cell(2) == 3 * 8 * 4
    # every row of every stencil against its members, per variable, FMA = 2 flops
    for (d, R), (sn, npts, nder, _, _) in bench._SHAPES.items():
        assert bench.contraction_flops_per_cell(d, R) == 2 * sn * (npts + nder) * (d + 2)
    assert bench.contraction_flops_per_cell(3, 2) == 34980
    # the FP64 reconstruction's figure contains the contraction
    for d, R in bench._SHAPES:
        assert bench.recon_flops_per_cell(d, R) > bench.contraction_flops_per_cell(d, R)


def test_profile_readers_follow_the_sources(tmp_path, monkeypatch):
    """The committed summary is read while its digest matches the sources; a
    summary whose digest differs (the kernel changed since) yields None."""
    kernel, workload = "k_recon_mixed", "3d_smooth_256"
    src = os.path.join(os.path.dirname(os.path.abspath(bench.__file__)), "profiles", f"{kernel}_{workload}.md")
    text = open(src).read()
    if f"sources digest: `{bench.sources_digest(kernel)}`" in text:
        assert bench.profiled_traffic(kernel, workload) > 0
        assert bench.profiled_figure(kernel, workload, "VALU instructions per wave") > 0
        assert bench.profiled_figure(kernel, workload, "waves per launch") == 256 ** 3 // 32
    else:
        # the kernel changed since the summary was taken: the bench reports null
        assert bench.profiled_traffic(kernel, workload) is None
    # the same readers against a copy of the tree whose summary carries another digest
    root = tmp_path / "tree"
    (root / "profiles").mkdir(parents=True)
    shutil.copytree(os.path.join(os.path.dirname(src), "..", "paper_2401_16543_amd", "csrc"),
                    root / "paper_2401_16543_amd" / "csrc")
    stale = text.replace(bench.sources_digest(kernel), "0" * 16)
    (root / "profiles" / f"{kernel}_{workload}.md").write_text(stale)
    monkeypatch.setattr(bench, "__file__", str(root / "bench.py"))
    assert bench.profiled_traffic(kernel, workload) is None
    assert bench.profiled_figure(kernel, workload, "VALU instructions per wave") is None
