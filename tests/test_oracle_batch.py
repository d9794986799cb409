"""Pins of the oracle's rate-distortion sweep."""

import numpy as np

from oracle import batch as OB
from oracle import codec as Co
from oracle import matrices as M
from synth import ar1_image


def test_sweep_entries_and_lossless_end():
    imgs = [ar1_image(16, 24, 0.95, seed=1), ar1_image(8, 8, 0.9, seed=2)]
    tab = OB.sse_table(imgs, ["T1", "DCT"], 1, 64)
    assert tab.shape == (2, 2, 64)
    assert np.all(tab[:, :, -1] == 0)                     # r = 64 reconstructs exactly
    assert tab[0, 0, 9] == Co.evaluate(imgs[0], M.T1, 10)["sse"]
    # r = 1: every transform whose first row is flat gives the block-mean image
    blocks = Co.to_blocks(imgs[1])
    mean = blocks.sum() / 64.0
    assert tab[1, 0, 0] == tab[1, 1, 0] == int(np.sum((blocks - np.rint(mean)) ** 2))


def test_mean_psnr_orders_transforms():
    imgs = [ar1_image(64, 64, 0.95, seed=s) for s in (3, 4)]
    tab = OB.sse_table(imgs, ["DCT", "T1", "LO"], 10, 10)
    p = OB.mean_psnr(tab, [im.shape for im in imgs])[:, 0]
    assert p[0] > p[1] > p[2]          # DCT above T1 above LO at r = 10 on AR(1) images
