"""Full reorthogonalisation on the GPU (kernel_flags bit 2; the remark of
Section 2.1 and the setting of every experiment of Section 5.1) against the
oracle's reorthogonalised APCG (``apcg(reorth=True)``), in FP64.

Per solve: the iteration count within +-2, the first CG coefficients to
1e-9, the true residual <= 1e-8; the Ritz values of the reorthogonalised
run are free of the repeated copies that a plain run produces (at most one
Ritz value within a relative 1e-10 of another), and the library's
selection at the paper's eps = 1e-14 equals the oracle's on the same
coefficients.  Over a sequence with the recycled basis (srks14): per system
+-2 iterations and +-2 columns."""
import numpy as np
import pytest

import gen
import oracle as O
from ritz_compare import selection_flips

pytestmark = pytest.mark.gpu


def _copies(th):
    t = np.sort(th)
    return int(np.sum(np.abs(np.diff(t)) <= 1e-10 * np.abs(t[1:])))


def test_reorth_solve_matches_oracle(gpu):
    import paper_1301_7530_amd as K

    seq = gen.config_elasticity(8, 1)
    rp, ci, v, b = seq.csr(0)
    ref = O.apcg(rp, ci, v, b, "block3", tol=1e-10, max_iter=3000, reorth=True)
    plain = O.apcg(rp, ci, v, b, "block3", tol=1e-10, max_iter=3000)
    s = K.sequence_for(gpu, seq, precision="fp64", reuse="selective", ritz_eps=1e-14, tol=1e-10, max_iter=3000,
                       reorth=True)
    try:
        s.submit(*seq.system(0))
        x, info = s.solve()
        a, r, _ = s.coeffs()
        s.recycle()
        th_lib, flags = s.ritz()
    finally:
        s.close()
    res = np.linalg.norm(b - O.spmv(rp, ci, v, x)) / np.linalg.norm(b)
    print(f"reorth: GPU {info['iters']} iterations, oracle {ref['m']} (without reorthogonalisation "
          f"{plain['m']}); rel res {res:.2e}", flush=True)
    assert info["status"] == 0 and res <= 1e-10 * 1.01
    assert abs(info["iters"] - ref["m"]) <= 2
    k = 40
    assert np.allclose(a[:k], ref["alpha"][:k], rtol=1e-9, atol=0)
    assert np.allclose(r[:k], ref["rho"][:k], rtol=1e-9, atol=0)
    th_m, th_m1 = O.ritz_values(a, r)
    th_p, _ = O.ritz_values(plain["alpha"], plain["rho"])
    print(f"Ritz copies: reorthogonalised {_copies(th_m)}, plain {_copies(th_p)}", flush=True)
    assert _copies(th_m) <= 1 < _copies(th_p)
    sel = np.nonzero(flags)[0]
    selection_flips(sel, O.srks_select(th_m, th_m1, 1e-14), th_m, th_m1, 1e-14)


def test_reorth_sequence_follows_oracle(gpu):
    import paper_1301_7530_amd as K

    seq = gen.config_elasticity(6, 4)
    eps = 1e-14
    recs, _ = O.solve_sequence(seq, 4, reuse="srks", eps=eps, tol=1e-8, max_iter=3000, reorth=True)
    s = K.sequence_for(gpu, seq, precision="fp64", reuse="selective", ritz_eps=eps, tol=1e-8, max_iter=3000,
                       reorth=True)
    got = []
    try:
        for k in range(4):
            s.submit(*seq.system(k))
            _, info = s.solve()
            assert info["status"] == 0 and info["rel_res_true"] <= 1e-8
            got.append((info["iters"], info["n_c"], s.recycle()))
    finally:
        s.close()
    want = [(q["m"], q["nc"], q["added"]) for q in recs]
    print("gpu   ", got, "\noracle", want, flush=True)
    for (m, nc, add), (mo, nco, addo) in zip(got, want):
        assert abs(m - mo) <= 2 and abs(nc - nco) <= 2 and abs(add - addo) <= 2


def test_reorth_rejected_outside_fp64(gpu):
    import paper_1301_7530_amd as K

    seq = gen.config_elasticity(4, 1)
    with pytest.raises(K.KrsError):
        K.sequence_for(gpu, seq, precision="fp32basis", reuse="selective", reorth=True)
