"""Helpers shared by the GPU tests: run the HIP path and compare it with the
oracle record by record."""
import numpy as np


def compare_results(got: dict, ref: dict, ids=None, f_rtol: float = 1e-12, label: str = ""):
    """got: sweep_to_numpy() of the HIP result; ref: oracle run_sets() dict.
    ids: for each oracle set, the index of that set in the HIP run."""
    S = ref["n_scales"]
    ns = ref["n_sets"]
    assert got["n_scales"] == S
    if ids is None:
        ids = np.arange(ns)
    bad = []
    for j in range(ns):
        for s in range(S):
            r = j * S + s
            q = int(ids[j]) * S + s
            a = got["members"][got["off"][q]:got["off"][q] + got["cnt"][q]]
            b = ref["members"][ref["off"][r]:ref["off"][r] + ref["cnt"][r]]
            if a.size != b.size or not np.array_equal(a, b):
                bad.append(("members", j, s, a.size, b.size))
            if got["K"][q] != ref["K"][r] or got["V"][q] != ref["V"][r]:
                bad.append(("KV", j, s, int(got["K"][q]), int(ref["K"][r]), int(got["V"][q]),
                            int(ref["V"][r])))
            if not np.array_equal(got["ctr"][q], ref["ctr"][r]):
                bad.append(("ctr", j, s, got["ctr"][q].tolist(), ref["ctr"][r].tolist()))
            fa, fb = float(got["f"][q]), float(ref["f"][r])
            if abs(fa - fb) > f_rtol * abs(fb):
                bad.append(("f", j, s, fa, fb))
            if len(bad) > 20:
                break
        if len(bad) > 20:
            break
    assert not bad, "%s: %d+ mismatches, first: %s" % (label, len(bad), bad[:8])
