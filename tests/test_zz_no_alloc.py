"""krs_seq_basis_noalloc (the allocation-free basis export) against
krs_seq_basis: the same columns bit for bit, on two calls in a row, the
second with a smaller sequence, in double precision and with a
single-precision basis (converted to double in the static scratch)."""
import ctypes

import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu


def _fill(K, ctx, seq, precision, systems):
    s = K.sequence_for(ctx, seq, precision=precision, reuse="selective", ritz_eps=1e-10, max_basis=24,
                       cap_policy="freeze", tol=1e-8, max_iter=5000)
    for k in range(systems):
        s.submit(*seq.system(k))
        _, info = s.solve()
        assert info["status"] == 0
        s.recycle()
    return s


@pytest.mark.parametrize("precision", ["fp64", "fp32basis"])
def test_basis_noalloc_equals_basis(gpu, precision):
    import paper_1301_7530_amd as K

    big = _fill(K, gpu, gen.config_elasticity(8, 2), precision, 2)
    small = _fill(K, gpu, gen.config_elasticity(5, 2), precision, 2)
    try:
        for s in (big, small):  # the second call has the smaller n
            ref = s.basis()
            got = s.basis_noalloc()
            print(f"{precision}: n={s.n} n_c={ref.shape[1]}", flush=True)
            assert ref.shape[1] > 0
            assert got.shape == ref.shape
            assert np.array_equal(got, ref)
        # the count-only form and a too-small output are reported like krs_seq_basis
        k = ctypes.c_int32(-1)
        assert K.lib().krs_seq_basis_noalloc(small.handle, None, small.n, 0, ctypes.byref(k)) == 0
        assert k.value == small.n_c
        out = np.zeros((small.n, 1), order="F")
        st = K.lib().krs_seq_basis_noalloc(small.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           small.n, 0, ctypes.byref(k))
        assert st == K.KRS_E_INVALID
    finally:
        big.close()
        small.close()


def test_basis_noalloc_rejects_n_beyond_scratch(gpu):
    import paper_1301_7530_amd as K

    seq = gen.make_sequence("diffusion", (164, 164, 164), 1, 1, 99)  # n = 4,410,944 > 4,194,304
    s = K.sequence_for(gpu, seq, precision="fp64", reuse="selective")
    try:
        k = ctypes.c_int32(-1)
        out = np.zeros((seq.n, 1), order="F")
        st = K.lib().krs_seq_basis_noalloc(s.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           seq.n, 1, ctypes.byref(k))
        assert st == K.KRS_E_INVALID
        assert b"4194304" in K.lib().krs_last_error()
    finally:
        s.close()
