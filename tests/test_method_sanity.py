"""Sanity of the method on a synthetic scene with known truth (not parity):
the oracle's reconstruction of the 160x120 one-plane scene removes the
dynamic rectangle (the refocused colour is the background's where the
reference shows the object) and finds the plane's disparity.  The paper has
no accuracy table; these bounds only catch a method that does not work."""
import numpy as np

import lf_scenes as S
import oracle as O
from lfcase import Case


def test_reconstruction_shows_the_background_behind_the_object():
    fr = S.make_frame(S.workload_spec("small"))
    c = Case.from_frame(fr, storage="f32")
    r = O.reconstruct(c.oracle_params(), c.views, c.S_P, c.mu_T, fr.spec.n_iters)
    # footprints beyond the frame edge are clamped: leave that band out
    band = int(np.ceil(max(abs(b) for b in c.baselines) * fr.disp_bg.max()))
    inner = np.zeros(fr.disp_bg.shape, bool)
    inner[:, band:-band] = True
    dyn = (fr.mask[c.ref] == 0) & inner
    err = np.abs(r["rgb"] - fr.bg_rgb).max(axis=-1)
    before = np.abs(c.views[c.ref].astype(np.float64) / 255 - fr.bg_rgb).max(axis=-1)
    assert np.median(before[dyn]) > 0.3                   # the object is really there
    assert np.median(err[dyn]) < 0.01 and (err[dyn] < 0.05).mean() > 0.6
    assert (err[~(fr.mask[c.ref] == 0) & inner] < 0.05).mean() > 0.95
    d = c.d_min + c.d_step * r["d_idx"]
    assert (np.abs(d - fr.disp_bg)[inner] <= 1).mean() > 0.97
