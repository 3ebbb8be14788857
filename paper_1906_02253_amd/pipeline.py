"""Host-side orchestration of the C-ABI calls for track finding: upload the
inputs, seed every track from its three seed hits (kf_seed), fit the three
seed hits (kf_fit), then find (kf_find).  Marshalling only."""
import numpy as np
import torch

from . import binding as B


class FindProblem:
    """Device-resident inputs of a finding run over many events."""

    def __init__(self, ctx, inp, prec=0, device="cuda"):
        self.ctx = ctx
        self.prec = prec
        self.hits = B.Hits(inp["x"], inp["y"], inp["z"], inp["su"], inp["sv"], inp["layer"], device)
        self.n_seeds = int(inp["seed_hits"].shape[0])
        self.ld = B.round_ld(self.n_seeds)
        ld = self.ld
        sh = np.full((3, ld), -1, np.int32)
        sh[:, :self.n_seeds] = inp["seed_hits"].T
        sl = np.full((3, ld), -1, np.int32)
        sl[:, :self.n_seeds] = inp["seed_layers"].T
        self.seed_hits = torch.as_tensor(sh, device=device)
        self.seed_layers = torch.as_tensor(sl, device=device)
        self.event_off = torch.as_tensor(inp["event_off"].astype(np.int32), device=device)
        se = np.zeros(ld, np.int32)
        se[:self.n_seeds] = inp["seed_event"]
        self.seed_event = torch.as_tensor(se, device=device)
        self.seeds = B.Tracks(self.n_seeds, ld, prec)
        self.out = B.Tracks(self.n_seeds, ld, prec)
        self.out_hits = torch.full((max(self.n_seeds, 1), ctx.n_layers), -1, dtype=torch.int32,
                                   device=device)
        # propagations, updates, chi2 tests, Newton evaluations, disk tests,
        # learned guesses, learned guesses that fell back
        self.counters = torch.zeros(B.N_COUNTERS, dtype=torch.int64, device=device)

    def seed_fit(self, flags=0):
        self.ctx.seed(self.hits, self.seed_hits, self.seeds, flags)
        self.ctx.fit(self.seeds, self.hits, self.seed_layers, self.seed_hits, 3, flags)

    def find(self, flags=0):
        self.ctx.find(self.hits, self.event_off, self.seeds, self.seed_event, self.seed_hits,
                      self.out_hits, self.out, self.counters, flags)

    def run(self, flags=0):
        self.seed_fit(flags)
        self.find(flags)

    def run_batched(self, flags=0):
        """The same pass as run(), as one captured graph (kf_find_batched)."""
        self.ctx.find_batched(self.hits, self.event_off, self.seed_hits, self.seed_layers,
                              self.seed_event, self.seeds, self.out_hits, self.out, self.counters,
                              flags)

    def autotune(self, flags=0, reps=3):
        return self.ctx.autotune(self.hits, self.event_off, self.seeds, self.seed_event,
                                 self.seed_hits, self.out_hits, self.out, flags, reps)

    def results(self):
        r = self.out.numpy()
        r["hits"] = self.out_hits[:self.n_seeds].cpu().numpy()
        r["counters"] = self.counters.cpu().numpy()
        return r
