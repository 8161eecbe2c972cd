"""Shared test helpers: seeded inputs on host and device, error bounds."""

from __future__ import annotations

import sys

import numpy as np

import synth

# Native work divisions the library exports (mg_num_tile_cfgs); every one is
# covered by the GPU parity tests.
NATIVE_CFGS = 30
# The last one is the naive one-output-per-lane mapping (no LDS, no MFMA).
NAIVE_CFG = 25
# Of those, the ones that load 16-byte aligned operands straight into LDS.
DMA_CFGS = (14, 15, 16, 17, 18, 19, 20, 21, 22, 23, 24, 26, 27, 28, 29)
# Of those, the ones with two k groups of wavefronts: each group sums half of
# every k-step and the halves are added at the end, a fixed order of its own
# (not the register-staged tiles' order, so not bit-identical to them).
KGROUP_CFGS = (26, 27, 28, 29)
# Split product-kernel work divisions (mg_split_num_cfgs), all covered likewise.
SPLIT_CFGS = 17

U64 = 2.0 ** -53  # unit roundoff of FP64
U32 = 2.0 ** -24


def host_mats(seed, m, n, k, kind="pm1"):
    A = synth.matrix(seed, synth.STREAM_A, m, k, kind=kind)
    B = synth.matrix(seed, synth.STREAM_B, k, n, kind=kind)
    C = synth.matrix(seed, synth.STREAM_C, m, n)
    return A, B, C


def to_dev(x, dtype=None, ld=None, fill=np.nan):
    """Host array -> CUDA tensor; with ``ld`` the rows are padded to ``ld``
    columns and the padding filled with ``fill`` (a view of the first cols
    is returned, keeping the padded parent alive through .base)."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    t = t.cuda()
    if ld is None or ld == x.shape[1]:
        return t
    big = torch.full((x.shape[0], ld), fill, dtype=t.dtype, device=t.device)
    big[:, : x.shape[1]] = t
    return big[:, : x.shape[1]]


def elementwise_bound(alpha, A, B, beta, C, k, u=U64):
    """Worst-case bound on |computed - exact| for any summation order with
    fused or unfused multiply-adds: (k + 2) u (|alpha| |A||B| + |beta||C|),
    plus a few ulps of the result."""
    absAB = np.abs(A) @ np.abs(B) if k > 0 else np.zeros((A.shape[0], B.shape[1]))
    mag = abs(alpha) * absAB + (abs(beta) * np.abs(C) if beta != 0 else 0.0)
    return (k + 2) * u * mag + 4 * u * np.abs(mag) + 1e-300


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def make_batch(seed, shapes, dtype=None, align=32, alpha=1.0, beta=1.0, device="cuda"):
    """Device operands for a batch: A, B, C of every problem carved from three
    flat U[-1,1) buffers at 256-byte aligned offsets.  Returns
    (views [(A, B, C)], flat buffers, problem descriptors)."""
    import torch
    import paper_1602_08477_amd as mg
    dtype = dtype or torch.float64
    offs = {"A": [], "B": [], "C": []}
    tot = {"A": 0, "B": 0, "C": 0}
    for m, n, k in shapes:
        for key, sz in (("A", m * k), ("B", k * n), ("C", m * n)):
            offs[key].append(tot[key])
            tot[key] += -(-sz // align) * align
    flats = {key: synth.flat_uniform(seed, i, max(tot[key], 1), device=device).to(dtype)
             for i, key in enumerate(("A", "B", "C"))}
    views, probs = [], []
    for i, (m, n, k) in enumerate(shapes):
        A = flats["A"][offs["A"][i]: offs["A"][i] + m * k].view(m, k)
        B = flats["B"][offs["B"][i]: offs["B"][i] + k * n].view(k, n)
        C = flats["C"][offs["C"][i]: offs["C"][i] + m * n].view(m, n)
        views.append((A, B, C))
        probs.append(mg.problem(A, B, C, alpha, beta))
    return views, flats, probs
