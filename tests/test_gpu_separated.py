"""GPU parity on a tile whose two 64-atom blocks lie just far enough apart to be
walked without the per-pair overlap test.

On such a separated tile every pair takes the non-overlapping form of the HCT
integral in both directions with y = (S/r)^2 <= 0.10, so the descreening and
chain walks evaluate only the short polynomial fits (and the FP32 chain walk
takes the factor (1 - y)^-2 of the derivatives from its fit instead of a
reciprocal).  Two compact clusters of 64 atoms are placed along x so that the
gap between their coordinate boxes just clears the separation rule (largest
pair y about 0.08, the upper part of the fits' range), and again 1.5 A closer,
where the same tile takes the tested walk.  The processing order is the
caller's (no reordering), so each cluster is one block.  Radii, energies,
forces, dE/dq and dE/drho are compared with the oracle at the tolerances of
the other parity tests, in both plans."""
import numpy as np
import pytest

import synth
from gpu_common import build, compare_system, gpu_eval, oracle_eval, params_pair

pytestmark = pytest.mark.gpu

OFFSET = 0.09          # IGB5 offset (A)
YFAR = 0.10            # the separated walk's limit on y


def _clusters(seed, closer=0.0):
    """Two 64-atom clusters (3.5 A globules) along x; returns the combined
    system and the host-side check of the separation rule for its two blocks
    (box gap against the screened radii, with the rule's margins)."""
    A = synth.make_system(seed, 64, 3.5)
    B = synth.make_system(seed + 1, 64, 3.5)
    xa = A.coords().astype(np.float64)
    xb = B.coords().astype(np.float64)
    xa -= xa.mean(0)
    xb -= xb.mean(0)
    SA, SB = A.screen * (A.rho - OFFSET), B.screen * (B.rho - OFFSET)
    ra, rb = (A.rho - OFFSET).max(), (B.rho - OFFSET).max()
    smax = max(SA.max(), SB.max())
    need = max(SB.max() + ra, SA.max() + rb) * 1.0001 + 1e-3
    gap = max(need, smax / np.sqrt(0.999 * YFAR)) * 1.002 - closer
    xb[:, 0] += xa[:, 0].max() - xb[:, 0].min() + gap
    xyz = synth.f32(np.concatenate([xa, xb]))
    cat = lambda a, b: np.concatenate([a, b])
    s = synth.System(xyz[:, 0].copy(), xyz[:, 1].copy(), xyz[:, 2].copy(), cat(A.q, B.q),
                     cat(A.rho, B.rho), cat(A.screen, B.screen))
    x32 = np.stack([s.x, s.y, s.z], 1).astype(np.float64)
    lo = [x32[:64].min(0), x32[64:].min(0)]
    hi = [x32[:64].max(0), x32[64:].max(0)]
    g = np.maximum(0.0, np.maximum(lo[1] - hi[0], lo[0] - hi[1]))
    g2 = float((g ** 2).sum())
    separated = g2 >= need ** 2 and smax ** 2 <= 0.999 * YFAR * g2
    r = np.sqrt(((x32[:64, None, :] - x32[None, 64:, :]) ** 2).sum(-1))
    ymax = float(max(((SB[None, :] / r) ** 2).max(), ((SA[:, None] / r) ** 2).max()))
    return s, separated, ymax


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("closer,expect_sep", [(0.0, True), (1.5, False)])
def test_cluster_pair_tile(prec, closer, expect_sep):
    s, separated, ymax = _clusters(11, closer)
    assert separated == expect_sep
    if expect_sep:
        assert 0.06 < ymax < YFAR                  # the upper part of the fits' range
    p_gpu, p_or = params_pair()
    _, batch, plan, atoms = build([s], prec)
    res = gpu_eval(plan, atoms, p_gpu)
    ref = oracle_eval(s, p_or)
    compare_system(res, 0, batch.atom_offset, ref, prec)
