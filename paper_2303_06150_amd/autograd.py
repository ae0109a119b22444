"""torch.autograd.Function over the library's moved-pose score and its adjoint.

RefineScore.apply(t, w, theta, pocket, poses) returns the trilinear score of
every pose of `poses` after the local move (t [n,3] translation, w [n,3]
axis-angle rotation about the pose's pivot, theta [total_torsions] bond angles,
torsions applied in reverse bond order).  Forward and backward are one lg_score
call (moves + gradient); this module only packs and unpacks the parameter layout
and applies the chain rule's upstream factor.
"""
from __future__ import annotations

import numpy as np
import torch

from . import lg


def move_layout(poses: lg.DeviceLigands):
    """Index tensors into the flat parameter layout 6 i + tors_offset[i]."""
    n = poses.n
    to = poses.tors_offset_host.astype(np.int64)
    base = 6 * np.arange(n, dtype=np.int64) + to[:-1]
    idx_t = (base[:, None] + np.arange(3)).reshape(-1)
    idx_w = (base[:, None] + 3 + np.arange(3)).reshape(-1)
    k = np.diff(to)
    pose_of_bond = np.repeat(np.arange(n, dtype=np.int64), k)
    idx_th = 6 * pose_of_bond + 6 + np.arange(int(to[-1]), dtype=np.int64)
    dev = poses.x.device
    as_t = lambda a: torch.from_numpy(a).to(dev)
    return as_t(idx_t), as_t(idx_w), as_t(idx_th), as_t(pose_of_bond), 6 * n + int(to[-1])


class RefineScore(torch.autograd.Function):
    @staticmethod
    def forward(ctx, t, w, theta, pocket, poses):
        idx_t, idx_w, idx_th, pose_of_bond, size = move_layout(poses)
        moves = torch.zeros(max(size, 1), dtype=torch.float32, device=t.device)
        moves[idx_t] = t.detach().reshape(-1).float()
        moves[idx_w] = w.detach().reshape(-1).float()
        moves[idx_th] = theta.detach().reshape(-1).float()
        res = lg.lg_score(pocket, poses, lg.LG_TRILINEAR, grad=True, moves=moves)
        ctx.save_for_backward(res["grad"])
        ctx.layout = (idx_t, idx_w, idx_th, pose_of_bond)
        ctx.n = poses.n
        return res["score"]

    @staticmethod
    def backward(ctx, g_score):
        (g,) = ctx.saved_tensors
        idx_t, idx_w, idx_th, pose_of_bond = ctx.layout
        n = ctx.n
        gs = g_score.reshape(n)
        gt = g[idx_t].reshape(n, 3) * gs[:, None]
        gw = g[idx_w].reshape(n, 3) * gs[:, None]
        gth = g[idx_th] * gs[pose_of_bond]
        return gt, gw, gth, None, None
