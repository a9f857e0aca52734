"""The particulate-suspension comparison of Sec. 6.1 (Table mutual) on a synthetic medium: a
100 x 100 image of non-touching 4 x 4 squares compressed into a 50 x 50 cell by annealing on S2,
on L2 of both phases, of the particles (w) and of the matrix (b), every result evaluated under
both descriptors.  The run is seeded and every step exact, so it is deterministic; the test
checks the paper's qualitative findings:
  - S2 compression gives by far the lowest S2 error and is also fair under L2;
  - L2 compression gives the lowest L2 error but an S2 error no better than a random image;
  - L2 of the matrix alone gives an S2 error worse than the random image;
  - the random image has the largest L2 error."""
from __future__ import annotations

import pytest

pytestmark = pytest.mark.gpu


def test_mutual_comparison_reproduces_paper_findings():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import bench
    from paper_1601_04359_amd import Context
    print("[gpu] mutual comparison 100x100 -> 50x50, 20000 steps x 4", flush=True)
    ctx = Context(0)
    rows, _ = bench.mutual_run(ctx, 20000, log=False)
    ctx.close()
    for k, v in rows.items():
        print(f"[gpu]   {k}: e(S2) {v['e_S2']:.4g}  e(L2) {v['e_L2']:.4g}", flush=True)
    eS = {k: v["e_S2"] for k, v in rows.items()}
    eL = {k: v["e_L2"] for k, v in rows.items()}
    assert min(eS, key=eS.get) == "S2" and eS["S2"] * 10 < eS["random"]
    assert eL["S2"] < 0.2 * eL["random"]
    assert min(eL, key=eL.get) == "L2" and eL["L2"] * 100 < eL["random"]
    assert eS["L2"] > 0.5 * eS["random"]
    assert eS["L2b"] > eS["random"]
    assert max(eL, key=eL.get) == "random"
