"""Helpers of the GPU parity tests: build a library context and the oracle's
view of the same seeded problem."""
from __future__ import annotations

import numpy as np

import synth
from oracle import csc, space as ospace, spinfree
from tests import layout


class Problem:
    """A seeded problem seen from both sides (oracle order and library layout)."""

    def __init__(self, ints, sp, seed=0):
        self.ints, self.sp = ints, sp
        if ints.spin_free:
            self.h, self.g = spinfree.expand(ints.h, ints.g)
        else:
            self.h, self.g = ints.h, ints.g
        self.cplx = ints.is_complex
        self.dets = ospace.enumerate_dets(sp.n_elec, sp.sub, sp.lo, sp.hi)
        self.perm = layout.Perm(self.dets, layout.layout_dets(sp.n_elec, sp.sub, sp.lo, sp.hi))
        self.seed = seed

    @classmethod
    def named(cls, name):
        ints, sp, _ = synth.config(name)
        cfg = synth.CONFIGS.get(name) or synth.TSPACES[name]
        return cls(ints, sp, cfg["seed"])

    def vector(self, seed=None):
        return synth.test_vector(len(self.dets), self.seed if seed is None else seed, complex_=self.cplx)

    def oracle_sigma(self, c, rows=None, nthreads=0):
        if rows is None:
            s = csc.sigma(self.dets, self.h, self.g, c, nthreads=nthreads)
        else:
            s = csc.sigma_rows(self.dets, self.h, self.g, c, rows, nthreads=nthreads)
        return s if self.cplx else s.real

    def context(self, device=0):
        import paper_2505_20375_amd as stpci
        ctx = stpci.Context(device)
        ctx.set_integrals(self.ints.h, self.ints.g, spin_free=self.ints.spin_free, e_core=self.ints.e_core)
        ctx.set_space(self.sp.n_elec, self.sp.sub, self.sp.lo, self.sp.hi)
        return ctx

    def to_device(self, x_oracle):
        import torch
        return torch.from_numpy(np.ascontiguousarray(self.perm.to_lib(x_oracle))).to("cuda")

    def from_device(self, t):
        return self.perm.to_oracle(t.cpu().numpy())


def rel_err(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)
