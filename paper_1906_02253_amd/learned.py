"""Host orchestration of the learned path-length guess: the training pairs'
targets come from the plain propagator (kf_propagate), the inputs from
kf_mlp_features, and the network is trained by kf_mlp_train.  Marshalling
only: every step runs in libkfmi.so."""
import numpy as np
import torch

from . import binding as B


def _tracks(states, prec):
    n = states.shape[0]
    t = B.Tracks(n, None, prec)
    t.par[:, :n] = torch.as_tensor(states.T, dtype=t.par.dtype)
    return t


class PairSet:
    """Device-resident training pairs: inputs [8, ld]; target [ld] the plain
    solve's path length minus the straight-line one in units of h s_line^2;
    and the rows where that solve succeeded."""

    def __init__(self, ctx, states, target_layer, prec=B.PREC_MIXED):
        n = states.shape[0]
        self.n = n
        self.states = states
        self.target_layer = torch.as_tensor(np.ascontiguousarray(target_layer, np.int32), device="cuda")
        t = _tracks(states, prec)
        self.ld = t.ld
        tl = torch.full((t.ld,), -1, dtype=torch.int32, device="cuda")
        tl[:n] = self.target_layer
        self.feats = torch.zeros((B.MLP_NIN, t.ld), dtype=torch.float32, device="cuda")
        ctx.mlp_features(t, tl, self.feats, prec)
        path = torch.zeros(t.ld, dtype=torch.float32, device="cuda")
        iters = torch.zeros(t.ld, dtype=torch.int32, device="cuda")
        ctx.propagate(t, tl, path, iters, flags=prec | B.NO_MATERIAL)
        # the correction to the straight-line path in units of h s_line^2
        self.target = torch.zeros(t.ld, dtype=torch.float32, device="cuda")
        ctx.mlp_targets(self.feats, path, n, self.target)
        self.path = path
        ok = (t.status[:n] == 0).cpu().numpy()
        self.ok_rows = np.nonzero(ok)[0].astype(np.int32)
        self.plain_iters = iters[:n].cpu().numpy()


def split_rows(rows, seed, frac=(0.9, 0.05, 0.05)):
    """Seeded split of row indices into train / validation / test."""
    rng = np.random.default_rng(seed)
    r = rows[rng.permutation(rows.shape[0])]
    a = int(frac[0] * r.shape[0])
    b = a + int(frac[1] * r.shape[0])
    return r[:a], r[a:b], r[b:]


def train(ctx, ps, train_rows, w0, epochs=20, batch=4096, lr=1e-3, seed=4):
    """Loads w0 and runs `epochs` passes of minibatch Adam over train_rows
    (shuffled per epoch with a seeded generator).  Returns the per-step
    losses (host)."""
    rng = np.random.default_rng(seed)
    ctx.mlp_load(w0)
    steps = train_rows.shape[0] // batch
    perm = np.concatenate([train_rows[rng.permutation(train_rows.shape[0])][:steps * batch]
                           for _ in range(epochs)]).astype(np.int32)
    rows = torch.as_tensor(perm, device="cuda")
    loss = torch.zeros(steps * epochs, dtype=torch.float32, device="cuda")
    ctx.mlp_train(ps.feats, ps.target, ps.n, rows, batch, steps * epochs, lr=lr, loss=loss)
    return loss.cpu().numpy()


def eval_loss(ctx, ps, rows):
    """Mean squared error of the network on `rows`."""
    r = torch.as_tensor(np.ascontiguousarray(rows, np.int32), device="cuda")
    g = torch.zeros(B.MLP_NPARAM, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    ctx.mlp_grad(ps.feats, ps.target, ps.n, r, g, loss)
    return float(loss.item())


def compare_starts(ctx, states, target_layer, prec=B.PREC_MIXED):
    """Propagates the same states with the plain and the learned start.
    Returns dict of (path, iters, status, par) for 'plain' and 'learned'."""
    n = states.shape[0]
    out = {}
    for name, flags in (("plain", 0), ("learned", B.INIT_MLP)):
        t = _tracks(states, prec)
        tl = torch.full((t.ld,), -1, dtype=torch.int32, device="cuda")
        tl[:n] = torch.as_tensor(np.ascontiguousarray(target_layer, np.int32), device="cuda")
        path = torch.zeros(t.ld, dtype=torch.float32, device="cuda")
        iters = torch.zeros(t.ld, dtype=torch.int32, device="cuda")
        ctx.propagate(t, tl, path, iters, flags=prec | B.NO_MATERIAL | flags)
        out[name] = dict(path=path[:n].cpu().numpy(), iters=iters[:n].cpu().numpy(),
                         status=t.status[:n].cpu().numpy(), par=t.par[:, :n].T.double().cpu().numpy())
    return out
