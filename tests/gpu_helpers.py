"""Shared helpers of the GPU tests: upload seeded inputs, run the library's
entry points through the C ABI and bring results back as numpy arrays.
No arithmetic of the method happens here."""
import numpy as np
import torch

import paper_0911_3191_amd as wd

DEV = torch.device("cuda:0")


class Setup:
    def __init__(self, dims, U, tap=True, precs=("fp64", "fp32", "i16", "f16"), recon=12, temporal=False):
        self.dims = tuple(dims)
        self.V = int(np.prod(dims))
        self.Vh = self.V // 2
        self.lat = wd.lattice(dims, tap)
        self.U = U
        self.gauge = wd.Gauge(self.lat, torch.from_numpy(np.ascontiguousarray(U)).to(DEV), precs, recon=recon,
                              temporal=temporal)

    def field(self, prec, nrhs=1):
        return wd.new_field(self.lat, prec, nrhs)

    def encode_full(self, prec, psi_full, parity, nrhs=1):
        """psi_full: numpy [nrhs?, V..., 4, 3, 2] -> encoded parity field."""
        f = self.field(prec, nrhs)
        canon = torch.from_numpy(np.ascontiguousarray(psi_full, dtype=np.float64)).to(DEV)
        wd.wd_spinor_encode_full(self.lat, prec, nrhs, parity, f, canon)
        torch.cuda.synchronize()
        return f

    def encode_parity(self, prec, psi_par, nrhs=1, basis=0):
        f = self.field(prec, nrhs)
        canon = torch.from_numpy(np.ascontiguousarray(psi_par, dtype=np.float64)).to(DEV)
        wd.wd_spinor_encode_basis(self.lat, prec, nrhs, basis, f, canon)
        torch.cuda.synchronize()
        return f

    def decode(self, prec, f, nrhs=1, basis=0):
        out = torch.zeros(nrhs * self.Vh * 24, dtype=torch.float64, device=DEV)
        wd.wd_spinor_decode_basis(self.lat, prec, nrhs, basis, out, f)
        torch.cuda.synchronize()
        a = out.cpu().numpy().reshape(nrhs, self.Vh, 4, 3, 2)
        return a[0] if nrhs == 1 else a


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))
