"""Helpers for GPU parity tests: move workload systems to the device, run the oracle."""
import numpy as np
import torch

from paper_2309_03060_amd import KronOperator, SystemSpec, decode_info

DEV = "cuda:0"


def to_spec(sys_):
    facs = [[torch.tensor(f, dtype=torch.float64, device=DEV) for f in row] for row in sys_.factors]
    diag = None if sys_.diag is None else torch.tensor(sys_.diag, dtype=torch.float64, device=DEV)
    return SystemSpec(factors=facs, sigma2=sys_.sigma2, diag=diag)


def make_op(systems, prec="fp32"):
    return KronOperator([to_spec(s) for s in systems], prec=prec)


def pack(arrs, dtype=torch.float64):
    return torch.cat([torch.tensor(np.asarray(a), dtype=dtype).reshape(-1) for a in arrs]).to(DEV).contiguous()


def unpack(t, systems, nrhs):
    out, off = [], 0
    v = t.detach().cpu().numpy().astype(np.float64)
    for s in systems:
        out.append(v[off:off + nrhs * s.n].reshape(nrhs, s.n))
        off += nrhs * s.n
    return out


def infos(info, count):
    return decode_info(info, count)


def rel_inf(got, ref):
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))
