"""Seeded multi-label Potts segmentation inputs (the multi-region extension of the binary energy).

Defines inputs only: integer data terms D[l, i] for every label l and pixel i, and integer Potts edge weights V on
the half-stencil layout of the binary energy (lambda folded in), plus the grid, stencil and block partition of the
binary DOPE solves that an expansion move runs.  None of the method's arithmetic lives here.

Image: a grey background (label 0) with nl - 1 random ellipses painted in order (ellipse l has label l, later ones
on top); region l has mean intensity (l + 0.5) / nl, plus N(0, sigma^2) noise.  D[l, i] = round(1000 (x_i - mu_l)^2
/ (2 sigma^2)) (Gaussian negative log-likelihood up to a constant, x1000); V = round(lam * 1000 exp(-dx^2 /
(2 sigma_w^2)) / |offset|) on the stencil.
"""
from __future__ import annotations

import dataclasses
from typing import Tuple

import numpy as np

from .configs import DEFAULT_MU0_2D, Problem, _round, _weights_from_features


@dataclasses.dataclass
class MultiLabelProblem:
    name: str
    template: Problem          # grid, stencil, block partition and ADMM schedule of the binary solves
    D: np.ndarray              # int32[nl, n]
    V: np.ndarray              # int32[h, n]
    truth: np.ndarray          # uint8[n] generating region of every pixel

    @property
    def n_labels(self) -> int:
        return int(self.D.shape[0])


def multilabel_image(seed: int = 0, W: int = 512, H: int = 512, n_labels: int = 4, conn: int = 8,
                     block: Tuple[int, int] = (32, 32), overlap: Tuple[int, int] = (2, 2), lam: float = 1.0,
                     sigma: float = 0.1, sigma_w: float = 0.1, mu0: int = DEFAULT_MU0_2D) -> MultiLabelProblem:
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:H, 0:W]
    region = np.zeros((H, W), dtype=np.uint8)
    for lab in range(1, n_labels):
        cx, cy = rng.uniform(0, W), rng.uniform(0, H)
        a, b = rng.uniform(0.1, 0.3) * W, rng.uniform(0.1, 0.3) * H
        th = rng.uniform(0, np.pi)
        dx, dy = xx - cx, yy - cy
        xr = dx * np.cos(th) + dy * np.sin(th)
        yr = -dx * np.sin(th) + dy * np.cos(th)
        region[(xr / a) ** 2 + (yr / b) ** 2 <= 1.0] = lab
    mus = (np.arange(n_labels) + 0.5) / n_labels
    img = mus[region] + rng.normal(0.0, sigma, size=(H, W))
    D = np.stack([_round(1000.0 * (img - m) ** 2 / (2.0 * sigma ** 2)).reshape(-1) for m in mus])
    V = _weights_from_features(img[None, :, :, None], 2, conn, sigma_w, scale=1000.0 * lam)
    template = Problem(f"multilabel{n_labels}_{W}x{H}_{conn}conn", (W, H, 1), 2, conn,
                       np.zeros(W * H, dtype=np.int32), np.zeros_like(V), 256, (block[0], block[1], 1),
                       (overlap[0], overlap[1], 0), mu0)
    return MultiLabelProblem(template.name, template, D.astype(np.int32), V.astype(np.int32),
                             region.reshape(-1).astype(np.uint8))
