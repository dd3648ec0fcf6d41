"""Shared set-up for the GPU parity tests: one synthetic ensemble handed to
both the oracle and the HIP library (through the C ABI)."""
import numpy as np

from oracle import dirac, subspace, coarse
from paper_2412_06347_amd import synth
from tests.gpu_util import to_dev, from_dev


class Pair:
    """Oracle objects and a GPU context built from the same seeded inputs."""

    def __init__(self, L, b, Nv, kappa=0.124, csw=1.0, eps=0.3, seed=1, Nlm=0, oracle_galerkin=True):
        import torch
        from paper_2412_06347_amd import mglma
        self.L, self.b, self.Nv, self.kappa = tuple(L), tuple(b), Nv, kappa
        self.U = synth.gauge_field(L, eps, seed)
        self.tv = synth.gaussian_fields(Nv, L, seed + 1000)
        self.D = dirac.WilsonClover(self.U, L, kappa, csw)
        self.bl = subspace.Blocking(L, b)
        self.B = subspace.BlockBasis(self.bl, dirac.fields_to_lattice(self.tv, L))
        self.nbr = self.bl.neighbour_table()
        self.D1 = coarse.galerkin(self.D, self.B) if oracle_galerkin else None
        self.ctx = mglma.Context(L, b, kappa, csw)
        self.ctx.load_gauge(to_dev(self.U))
        tvd = self.fine_dev(self.tv)
        self.ctx.build_subspace(tvd)
        self.top = None
        if Nlm:
            self.modes = synth.gaussian_coarse(Nlm, self.bl.V1, 2 * Nv, seed + 2000)
            self.top = coarse.TopLevel(self.modes, self.D1, self.nbr, Nv)
            self.ctx.set_top_modes(to_dev(self.modes))
        torch.cuda.synchronize()

    # canonical numpy <-> device layout through the ABI converters
    def fine_dev(self, canon, prec=0):
        x = self.ctx.fine(canon.shape[0], prec)
        self.ctx.import_fields(to_dev(canon), x, prec)
        return x

    def fine_host(self, dev, prec=0):
        import torch
        out = torch.empty((dev.shape[0], self.ctx.V, 4, 3, 2), dtype=torch.float64, device="cuda")
        self.ctx.export_fields(dev, out, prec)
        return from_dev(out)

    def lat(self, canon):
        return dirac.fields_to_lattice(canon, self.L)

    def canon(self, lat):
        return dirac.fields_to_canonical(lat)
