"""CPU-only checks of the C-ABI library: it loads, exports every function the
header declares, and rejects invalid arguments before touching a GPU."""
import ctypes as C

import pytest

from paper_2112_03851_amd import sos


def test_library_exports_every_declared_symbol():
    L = sos.lib()
    names = sos.declared_functions()
    assert "sos_setup" in names and "sos_solve" in names and "sos_last_error" in names
    for n in names:
        assert hasattr(L, n), n
    raw = C.CDLL(sos.LIB_PATH)
    for n in names:
        getattr(raw, n)


def test_opts_defaults():
    o = sos.default_opts(sos.SOS_FP64)
    assert o.precision == sos.SOS_FP64 and o.mode == sos.SOS_STEPWISE
    assert o.inner_abs == 1e-10 and o.inner_tol == 0.0 and o.G == 6.672e-11
    o = sos.default_opts(sos.SOS_FP32_INNER)
    assert o.mode == sos.SOS_BATCHED and o.inner_tol == 1e-2 and o.use_graph == 1
    assert o.wave_rows == 0 and o.resident == 1 and o.block == 0 and o.team == 0


@pytest.mark.parametrize("kw,msg", [
    (dict(ne=(4, 4, 4), cuts=((2, 2), (), ())), "cuts"),
    (dict(ne=(4, 4, 4), cuts=((0,), (), ())), "cuts"),
    (dict(ne=(4, 4, 4), cuts=((4,), (), ())), "cuts"),
    (dict(ne=(4, 4, 4), nparts=(3, 1, 1)), "equal split"),
    (dict(ne=(0, 4, 4), nparts=(1, 1, 1)), "ne"),
    (dict(ne=(4, 4, 4), nparts=(2, 1, 1), p=-1.0), "Robin"),
    (dict(ne=(4, 4, 4), nparts=(2, 1, 1), p=float("nan")), "Robin"),
    (dict(ne=(4, 4, 4), nparts=(2, 1, 1), bc=(1,) * 6), "Dirichlet"),
    (dict(ne=(4, 4, 4), lengths=(1.0, -1.0, 1.0), nparts=(2, 1, 1)), "len"),
    (dict(ne=(4, 4, 4), nparts=(2, 1, 1), max_outer=0), "max_outer"),
    (dict(ne=(4, 4, 4), nparts=(2, 1, 1), check_every=0), "check_every"),
    (dict(ne=(4, 4, 4), nparts=(2, 1, 1), block=100), "block"),
    (dict(ne=(4, 4, 4), nparts=(2, 1, 1), inner_tol=0.0, inner_abs=0.0), "inner_tol"),
    (dict(ne=(4, 4, 4), nparts=(2, 1, 1), copies=0), "copies"),
    (dict(ne=(4, 4, 4), nparts=(2, 1, 1), copies=5000), "copies"),
    (dict(ne=(4, 4, 4), nparts=(2, 1, 1), copies=3, p=[1.0, 0.0, 2.0]), "Robin"),
    (dict(ne=(4, 4, 4), nparts=(2, 1, 1), copies=2, p=1.0, q=[0.0, -1.0]), "second-order"),
    (dict(ne=(4, 4, 4), nparts=(2, 1, 1), wave_rows=1), "wave_rows"),
    (dict(ne=(4, 4, 4), nparts=(2, 1, 1), block=256, wave_rows=2), "wave_rows"),
    (dict(ne=(4, 4, 4), nparts=(2, 1, 1), resident=3), "resident"),
    (dict(ne=(4, 4, 4), nparts=(2, 1, 1), team=9), "team"),
])
def test_invalid_arguments_rejected_on_the_host(kw, msg):
    with pytest.raises(sos.SosError) as ei:
        sos.Problem(**kw)
    assert ei.value.code == sos.SOS_EINVAL
    assert msg in str(ei.value)


def test_per_face_robin_values_checked():
    with pytest.raises(sos.SosError) as ei:
        sos.Problem((4, 4, 4), nparts=(2, 1, 1), p=[1.0, 0.0])
    assert ei.value.code == sos.SOS_EINVAL
    with pytest.raises(ValueError):
        sos.Problem((4, 4, 4), nparts=(2, 2, 1), p=[1.0, 1.0])
    assert sos.Problem._count_faces([4, 4, 4]) == 288
    assert sos.Problem._count_faces([16, 16, 1]) == 960
    assert sos.Problem._count_faces([8, 8, 8]) == 2688
