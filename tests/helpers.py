"""Shared checks of GPU results against the oracle (imported by the GPU test
modules; not a test module itself)."""
import numpy as np

from oracle import c_oracle


def sampled_checks(w, gpu, rows):
    """Exact per-row checks against the oracle at any size."""
    lab, core, cnt = gpu[:3]
    n = w.n
    assert (core == (cnt >= w.minpts)).all()
    ref_cnt = c_oracle.row_counts(w.points, w.eps, rows)
    np.testing.assert_array_equal(cnt[rows], ref_cnt)
    # canonical labels everywhere
    nz = lab >= 0
    assert (lab >= -1).all()
    assert core[lab[nz]].all()
    assert (lab[lab[nz]] == lab[nz]).all()
    ci = np.flatnonzero(core)
    assert (lab[ci] <= ci).all() and (lab[ci] >= 0).all()
    # per sampled row: neighbours, their exact core flags, label rules
    for i in rows[:4]:
        nb = np.flatnonzero(c_oracle.row_neighbours(w.points, w.eps, int(i)))
        nb_core = c_oracle.row_counts(w.points, w.eps, nb) >= w.minpts
        np.testing.assert_array_equal(core[nb], nb_core)
        core_nb = nb[nb_core]
        if core[i]:
            assert (lab[core_nb] == lab[i]).all()
        elif core_nb.size:
            assert lab[i] == lab[core_nb.min()]
        else:
            assert lab[i] == -1
    assert n == len(lab)
