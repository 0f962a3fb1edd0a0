"""ddhf_detect_noalloc (fixed scratch array, no workspace) against ddhf_detect
with a caller workspace: mask, labels, boxes and counts bit for bit, on two
calls in a row, the second on a smaller frame (the scratch then holds the
first call's leftovers), and both against the oracle's detection."""
import numpy as np
import pytest
import torch

import oracle
from paper_2603_08386_amd import ddhf as D
from paper_2603_08386_amd.synth import Grid, Params

from gpu_common import DEV, banner

pytestmark = pytest.mark.gpu


def scene(W, H, seed, density):
    rng = np.random.default_rng(seed)
    counts = rng.integers(0, 12, size=W * H)
    row_ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    active = np.flatnonzero(counts >= 6).astype(np.int32)
    on = rng.random(active.size) < density
    sf = np.where(on, rng.uniform(0.1, 0.85, active.size), rng.uniform(0.3, 1.0, active.size))
    snr = np.where(on, rng.uniform(1.5, 9.0, active.size), rng.uniform(0.0, 3.0, active.size))
    b = rng.integers(0, 3981, size=active.size).astype(np.int32)
    return active, row_ptr, sf.astype(np.float32), snr.astype(np.float32), b


def call(fn, inputs, W, H, grid, prm, max_boxes=512):
    active, row_ptr, sf, snr, b = (torch.from_numpy(np.ascontiguousarray(a)).to(DEV) for a in inputs)
    na = int(active.numel())
    mask = torch.full((W * H,), 7, dtype=torch.uint8, device=DEV)
    labels = torch.full((W * H,), 7, dtype=torch.int32, device=DEV)
    boxes = torch.zeros(max_boxes * 32, dtype=torch.uint8, device=DEV)
    nb = torch.full((2,), -5, dtype=torch.int32, device=DEV)
    args = (active, row_ptr, sf, snr, b, na, W, H, D.make_grid(grid), D.make_params(prm), mask,
            labels, boxes, max_boxes, nb)
    if fn == "ws":
        D.ddhf_detect(*args, D.workspace(D.ddhf_detect_workspace_size(W, H), DEV))
    else:
        D.ddhf_detect_noalloc(*args)
    torch.cuda.synchronize()
    n = int(nb[0].item())
    return (mask.cpu().numpy(), labels.cpu().numpy(), D.boxes_to_list(boxes, min(n, max_boxes)),
            n, int(nb[1].item()))


def test_noalloc_matches_workspace_entry_point_twice():
    grid = Grid(f0=10_000, df=500, K=3981)
    prm = Params(a_min=16, alpha=0.5)
    # second call: a smaller frame; both stay under the 1024 merge candidates
    cases = [(320, 240, 11, 0.45), (200, 120, 12, 0.45)]
    for W, H, seed, dens in cases:
        banner(f"detect_noalloc {W}x{H}")
        inputs = scene(W, H, seed, dens)
        ref = call("ws", inputs, W, H, grid, prm)
        got = call("noalloc", inputs, W, H, grid, prm)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
        assert got[2] == ref[2] and got[3:] == ref[3:]
        assert ref[3] > 10 and ref[4] == 0
        active, row_ptr, sf, snr, b = inputs
        tau = Params(**{**prm.__dict__})
        tau.tau_sf, tau.tau_comb = float(np.float32(prm.tau_sf)), float(np.float32(prm.tau_comb))
        tau.alpha = float(np.float32(prm.alpha))
        m64, lab64, boxes64, n64 = oracle.detect(active, row_ptr, sf.astype(np.float64),
                                                 snr.astype(np.float64), b, W, H, grid, tau)
        assert np.array_equal(got[0], m64) and np.array_equal(got[1], lab64) and got[3] == n64
        for g1, o1 in zip(got[2], boxes64):
            for k in ["x0", "y0", "x1", "y1", "n_px", "rep_pixel"]:
                assert g1[k] == o1[k]


def test_noalloc_refuses_frames_above_its_limit():
    grid = Grid(f0=10_000, df=500, K=3981)
    z = torch.zeros(16, dtype=torch.int32, device=DEV)
    with pytest.raises(D.DdhfError) as e:
        D.ddhf_detect_noalloc(z, z, z, z, z, 0, 2048, 1024, D.make_grid(grid),
                              D.make_params(Params()), z, z, z, 1, z)
    assert e.value.status == D.DDHF_ENOSPACE
