"""Write problems (concatenated as independent instances) in the binary format
read by tests/host/plan_check.cpp."""
import numpy as np


def dump_problems(problems, path, values=False):
    rp = [0]
    ci, part, sop = [], [], []
    M = N = NP = 0
    for k, p in enumerate(problems):
        rp += (p.indptr[1:].astype(np.int64) + rp[-1]).tolist()
        ci.append(p.indices.astype(np.int64) + N)
        part.append(p.part.astype(np.int64) + NP)
        sop += [k] * p.nparts
        M += p.m; N += p.n; NP += p.nparts
    ci = np.concatenate(ci).astype(np.int32)
    part = np.concatenate(part).astype(np.int32)
    with open(path, "wb") as f:
        np.array([M, N, len(ci), NP, len(problems)], dtype=np.int32).tofile(f)
        np.array(rp, dtype=np.int32).tofile(f)
        ci.tofile(f)
        part.tofile(f)
        np.array(sop, dtype=np.int32).tofile(f)
        if values:
            np.concatenate([np.asarray(p.data, dtype=np.float64) for p in problems]).tofile(f)
