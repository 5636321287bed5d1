"""Host-side tests of the C ABI that need no GPU: the library loads and exports
every function include/tlib.h declares, descriptors are validated with the
documented error codes, layouts give the paper's strides, and the planner
(in plan-only mode, which launches nothing and touches no device memory)
collapses problems into the expected kernels."""
import ctypes
import os
import re

import pytest

import paper_1711_10912_amd as T
from paper_1711_10912_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = 1 << 40  # never dereferenced: plan-only mode


def _declared():
    src = open(os.path.join(ROOT, "include", "tlib.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tlib_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    names = _declared()
    assert "tlib_ttv" in names and "tlib_ttt" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib.EXPORTS)
    assert b"gfx950" in L.tlib_version()


def test_strides_from_layout_matches_paper():
    assert T.strides((4, 2, 3)) == (1, 4, 8)
    assert T.strides((4, 2, 3), (3, 2, 1)) == (6, 3, 1)
    assert T.strides((4, 3, 2), (1, 2, 3)) == (1, 4, 12)
    with pytest.raises(_lib.TlibError) as e:
        T.strides((2, 3), (1, 1))
    assert e.value.code == _lib.EMODE


class Plan:
    def __enter__(self):
        _lib.lib().tlib_set_plan_only(1)
        return self

    def __exit__(self, *a):
        _lib.lib().tlib_set_plan_only(0)


def _d(shape, dtype=_lib.F64, layout=None, strides=None, ptr=FAKE):
    return _lib.desc(ptr, dtype, shape, strides, layout)


def _ttv(A, b, m, C):
    return _lib.lib().tlib_ttv(ctypes.byref(A), ctypes.byref(b), m, ctypes.byref(C), None)


def _ttm(A, B, m, C):
    return _lib.lib().tlib_ttm(ctypes.byref(A), ctypes.byref(B), m, ctypes.byref(C), None)


def _plan():
    return _lib.lib().tlib_last_plan().decode()


def test_ttv_regimes():
    with Plan():
        n = 406
        A = _d((n, n, n), ptr=FAKE)
        b = _d((n,), ptr=FAKE * 2)
        C = _d((n, n), ptr=FAKE * 3)
        # mode 1: every output a contiguous fiber of 406
        assert _ttv(A, b, 1, C) == 0 and _plan().startswith("ttv fiber")
        assert _ttv(A, b, 2, C) == 0 and _plan().startswith("ttv col") and "n_lo=406" in _plan()
        assert _ttv(A, b, 3, C) == 0 and _plan().startswith("ttv col") and "n_lo=164836" in _plan()
        # last-order A: mode 3 is the stride-1 mode
        A = _d((n, n, n), layout=(3, 2, 1))
        Cl = _d((n, n), layout=(2, 1), ptr=FAKE * 3)
        assert _ttv(A, b, 3, Cl) == 0 and _plan().startswith("ttv fiber")
        # short contiguous fibers (20 < 32) are staged through slabs
        A20 = _d((20,) * 4)
        b20 = _d((20,), ptr=FAKE * 2)
        C20 = _d((20,) * 3, ptr=FAKE * 3)
        assert _ttv(A20, b20, 1, C20) == 0 and _plan().startswith("ttv slab")
        # a workgroup's slabs span whole 16-byte units (13^7, mode 1: 52-byte
        # FP32 slabs in multiples of four), so every run is copied with
        # 16-byte loads
        for dt, es in ((_lib.F32, 4), (_lib.F64, 8)):
            A13 = _d((13,) * 7, dt)
            b13 = _d((13,), dt, ptr=FAKE * 2)
            C13 = _d((13,) * 6, dt, ptr=FAKE * 3)
            assert _ttv(A13, b13, 1, C13) == 0 and _plan().startswith("ttv slab")
            slabs = int(re.search(r"slabs=(\d+)", _plan()).group(1))
            assert slabs > 1 and (slabs * 13 * es) % 16 == 0, _plan()
        # n_lo of 32..63: whole dense slabs (36^5, mode 2) go to the slab
        # kernel; slabs too long for it (37x600, three of them) or a lo with
        # gaps stay on the col kernel
        A36 = _d((36,) * 5)
        b36 = _d((36,), ptr=FAKE * 2)
        C36 = _d((36,) * 4, ptr=FAKE * 3)
        assert _ttv(A36, b36, 2, C36) == 0 and _plan().startswith("ttv slab") and "n_lo=36" in _plan()
        Ak = _d((37, 600, 3))
        bk = _d((600,), ptr=FAKE * 2)
        Ck = _d((37, 3), ptr=FAKE * 3)
        assert _ttv(Ak, bk, 2, Ck) == 0 and _plan().startswith("ttv col") and "ksplit=" in _plan()
        Ag = _d((40, 30, 3000), strides=(2, 80, 2400))
        bg = _d((30,), ptr=FAKE * 2)
        Cg = _d((40, 3000), ptr=FAKE * 3)
        assert _ttv(Ag, bg, 2, Cg) == 0 and _plan().startswith("ttv col") and "n_lo=40" in _plan()
        # a C layout that does not follow A's: the dims do not merge, short lo
        # (13 < 32): one fiber per output
        A = _d((13,) * 4)
        b = _d((13,), ptr=FAKE * 2)
        C = _d((13,) * 3, layout=(3, 1, 2), ptr=FAKE * 3)
        assert _ttv(A, b, 2, C) == 0 and _plan().startswith("ttv fiber")
        # a view with gaps (every other index of mode 1, trimmed mode 2): col
        # kernel with the hi index over two dims
        Av = _d((64, 30, 20), strides=(2, 200, 10000))
        bv = _d((20,), ptr=FAKE * 2)
        Cv = _d((64, 30), ptr=FAKE * 3)
        assert _ttv(Av, bv, 3, Cv) == 0 and _plan().startswith("ttv col") and "hidims=1" in _plan()
        # five output dims that merge with nothing: generic kernel
        A6 = _d((3, 4, 5, 6, 7, 2))
        b6 = _d((3,), ptr=FAKE * 2)
        C6 = _d((4, 5, 6, 7, 2), layout=(5, 4, 3, 2, 1), ptr=FAKE * 3)
        assert _ttv(A6, b6, 1, C6) == 0 and _plan().startswith("ttv generic")


def test_ttm_and_ttt_plans():
    with Plan():
        A = _d((90, 90, 90, 90), _lib.F32)
        B = _d((64, 90), _lib.F32, ptr=FAKE * 2)
        C = _d((90, 64, 90, 90), _lib.F32, ptr=FAKE * 3)
        assert _ttm(A, B, 2, C) == 0
        p = _plan()
        assert "gemm" in p and "M=64" in p and "K=90" in p and "N=729000" in p
        Ad = _d((96, 80, 64, 48), _lib.BF16, layout=(3, 1, 4, 2))
        Bd = _d((64, 48, 120), _lib.BF16, ptr=FAKE * 2)
        Cd = _d((96, 80, 120), _lib.F32, ptr=FAKE * 3)
        phi = _lib.i32_array((1, 2, 3, 4))
        psi = _lib.i32_array((3, 1, 2))
        rc = _lib.lib().tlib_ttt(ctypes.byref(Ad), ctypes.byref(Bd), 2, phi, psi, ctypes.byref(Cd), None)
        assert rc == 0
        p = _plan()
        # C is first-order, so its unit-stride mode (free A mode 1) becomes the GEMM's N side
        assert "M=120" in p and "N=7680" in p and "K=3072" in p and "dims=(1,2,2)" in p


def test_first_order_ttt_collapses_to_plain_gemm():
    with Plan():
        Ad = _d((96, 80, 64, 48), _lib.F32)
        Bd = _d((64, 48, 120), _lib.F32, ptr=FAKE * 2)
        Cd = _d((96, 80, 120), _lib.F32, ptr=FAKE * 3)
        rc = _lib.lib().tlib_ttt(ctypes.byref(Ad), ctypes.byref(Bd), 2, _lib.i32_array((1, 2, 3, 4)),
                                 _lib.i32_array((3, 1, 2)), ctypes.byref(Cd), None)
        assert rc == 0 and "dims=(1,1,1)" in _plan()


def _ksplit(plan):
    return int(plan.split("ksplit=")[1].split()[0])


def test_ttt_noalloc_bounds_its_split_by_the_static_scratch():
    """tlib_ttt_noalloc plans the same contraction as tlib_ttt (Sec. 5.2
    Eq. ttt) with its split-K slices bounded by the static scratch size."""
    L = _lib.lib()
    cap = 16 << 20
    with Plan():
        for (na, nb, nc, dt, es) in (((96, 80, 64, 48), (64, 48, 120), (96, 80, 120), _lib.F32, 4),  # 3.7 MB a slice
                                     ((8, 4, 4096), (4, 4096, 8), (8, 8), _lib.F32, 4),  # tiny M N, deep K
                                     ((1500, 512), (512, 1500), (1500, 1500), _lib.F64, 8)):  # a slice > cap
            Ad = _d(na, dt)
            Bd = _d(nb, dt, ptr=FAKE * 2)
            Cd = _d(nc, dt, ptr=FAKE * 3)
            q = (len(na) + len(nb) - len(nc)) // 2
            phi = _lib.i32_array(tuple(range(1, len(na) + 1)))
            psi = _lib.i32_array(tuple(range(q + 1, len(nb) + 1)) + tuple(range(1, q + 1)))
            assert L.tlib_ttt(ctypes.byref(Ad), ctypes.byref(Bd), q, phi, psi, ctypes.byref(Cd), None) == 0
            ref = _plan()
            assert L.tlib_ttt_noalloc(ctypes.byref(Ad), ctypes.byref(Bd), q, phi, psi, ctypes.byref(Cd), None) == 0
            got = _plan()
            mn = 1
            for e in nc:
                mn *= e
            assert _ksplit(got) <= max(1, cap // (es * mn)), got
            if es * mn > cap:
                assert _ksplit(ref) > 1 and _ksplit(got) == 1
            assert _ksplit(got) <= _ksplit(ref)
            # everything but the split is the same plan
            strip = lambda p: p.split(" ksplit=")[0]
            assert strip(got) == strip(ref)
        # the same errors as tlib_ttt
        Ad = _d((3, 4, 2, 6))
        Cd = _d((2, 3, 4), ptr=FAKE * 2)
        Ed = _d((3, 6, 3), ptr=FAKE * 3)
        assert L.tlib_ttt_noalloc(ctypes.byref(Ad), ctypes.byref(Cd), 2, _lib.i32_array((1, 4, 3, 2)),
                                  _lib.i32_array((2, 3, 1)), ctypes.byref(Ed), None) == _lib.ESHAPE
        assert L.tlib_ttt_noalloc(ctypes.byref(Ad), ctypes.byref(Cd), 2, _lib.i32_array((1, 1, 2, 3)),
                                  _lib.i32_array((2, 3, 1)), ctypes.byref(Ed), None) == _lib.EMODE


def test_error_codes():
    with Plan():
        A = _d((4, 5, 6))
        b = _d((5,), ptr=FAKE * 2)
        C = _d((4, 6), ptr=FAKE * 3)
        assert _ttv(A, b, 2, C) == 0
        assert _ttv(A, b, 4, C) == _lib.EMODE
        assert _ttv(A, b, 0, C) == _lib.EMODE
        assert _ttv(A, _d((6,), ptr=FAKE * 2), 2, C) == _lib.ESHAPE
        assert _ttv(A, b, 2, _d((4, 7), ptr=FAKE * 3)) == _lib.ESHAPE
        assert _ttv(A, _d((5,), _lib.F32, ptr=FAKE * 2), 2, C) == _lib.EDTYPE
        assert _ttv(A, b, 2, _d((4, 6), _lib.F32, ptr=FAKE * 3)) == _lib.EDTYPE
        assert _ttv(_d((4,)), _d((4,), ptr=FAKE * 2), 1, _d((), ptr=FAKE * 3)) == _lib.EINVAL
        assert _ttv(A, b, 2, _d((4, 6), ptr=FAKE + 8)) == _lib.EALIAS
        assert _ttv(A, b, 2, _d((4, 6), strides=(1, 2), ptr=FAKE * 3)) == _lib.ESTRIDE
        assert _ttv(A, b, 2, _d((4, 6), strides=(-1, 4), ptr=FAKE * 3)) == _lib.EINVAL
        assert _ttv(_d((4, 0, 6)), b, 2, C) == _lib.EINVAL
        assert _ttv(A, b, 2, _d((4, 6), layout=(1, 1), ptr=FAKE * 3)) == _lib.EMODE
        assert _ttv(_d((4, 5, 6), dtype=7), b, 2, C) == _lib.EDTYPE
        assert b"mode" in _lib.lib().tlib_last_error() or True
        # TTT: pairs with unequal extents, bad permutations
        Ad = _d((3, 4, 2, 6))
        Cd = _d((2, 3, 4), ptr=FAKE * 2)
        Ed = _d((3, 6, 3), ptr=FAKE * 3)
        L = _lib.lib()
        ok = L.tlib_ttt(ctypes.byref(Ad), ctypes.byref(Cd), 2, _lib.i32_array((1, 4, 2, 3)),
                        _lib.i32_array((2, 3, 1)), ctypes.byref(Ed), None)
        assert ok == 0  # the paper's times_tensor example E: shape (3,6,3)
        bad = L.tlib_ttt(ctypes.byref(Ad), ctypes.byref(Cd), 2, _lib.i32_array((1, 4, 3, 2)),
                         _lib.i32_array((2, 3, 1)), ctypes.byref(Ed), None)
        assert bad == _lib.ESHAPE
        bad = L.tlib_ttt(ctypes.byref(Ad), ctypes.byref(Cd), 2, _lib.i32_array((1, 1, 2, 3)),
                         _lib.i32_array((2, 3, 1)), ctypes.byref(Ed), None)
        assert bad == _lib.EMODE
        # add in place is allowed only on the very same view
        X = _d((10, 10), _lib.F32)
        Y = _d((10, 10), _lib.F32, ptr=FAKE * 2)
        assert L.tlib_add(1.0, ctypes.byref(X), 1.0, ctypes.byref(Y), ctypes.byref(X), None) == 0
        Xt = _d((10, 10), _lib.F32, layout=(2, 1))
        assert L.tlib_add(1.0, ctypes.byref(X), 1.0, ctypes.byref(Y), ctypes.byref(Xt), None) == _lib.EALIAS


def test_error_message_names_the_problem():
    with Plan():
        A = _d((4, 5, 6))
        rc = _ttv(A, _d((6,), ptr=FAKE * 2), 2, _d((4, 6), ptr=FAKE * 3))
        assert rc == _lib.ESHAPE
        assert b"n_2" in _lib.lib().tlib_last_error()
        assert _lib.lib().tlib_strerror(_lib.ESHAPE) == b"shape mismatch"


def test_binding_refuses_cpu_tensors():
    import torch
    A = torch.zeros(3, 4)
    with pytest.raises(_lib.TlibError):
        T.ttv(A, torch.zeros(4), 2)


def test_autotune_controls(tmp_path):
    """Autotune mode switch, table save/load round trip and load errors
    (no GPU: plan-only calls never tune)."""
    import paper_1711_10912_amd as T
    L = _lib.lib()
    assert L.tlib_set_autotune(7) == -1          # unknown mode: unchanged
    prev = T.set_autotune("frozen")
    try:
        assert T.set_autotune("on") == "frozen"
        T.autotune_clear()
        assert T.autotune_entries() == 0
        tab = tmp_path / "tab.txt"
        tab.write_text("2 ttm|2|0:3,4/1,5/4,6/20|0:2,7/1,4/7|0:3,4/1,7/4,6/28\n"
                       "5 ttt|1|1|2|1|2|1:2,3/1,4/3|1:2,4/1,2/4|1:2,3/1,2/3\n")
        T.autotune_load(str(tab))
        assert T.autotune_entries() == 2
        out = tmp_path / "out.txt"
        T.autotune_save(str(out))
        assert sorted(out.read_text().splitlines()) == sorted(tab.read_text().splitlines())
        bad = tmp_path / "bad.txt"
        bad.write_text("3 ok|line\nnot-a-number key\n")
        with pytest.raises(T.TlibError):
            T.autotune_load(str(bad))
        assert T.autotune_entries() == 3           # the good line before the bad one is kept
        with pytest.raises(T.TlibError):
            T.autotune_load(str(tmp_path / "missing.txt"))
    finally:
        T.autotune_clear()
        T.set_autotune(prev)


def test_autotune_class_entries_serve_unseen_shapes(tmp_path):
    """A table entry keyed by shape class (dtype, layout flags, base-4 size
    buckets) serves shapes that have no exact entry; an exact entry wins over
    its class's (plan-only calls in frozen mode never tune)."""
    import paper_1711_10912_amd as T
    prev = T.set_autotune("frozen")
    try:
        T.autotune_clear()
        tab = tmp_path / "cls.txt"
        # TTM FP32, mode 2 not unit-stride, C not contiguous along j, n_m 90
        # (bucket 3), 64 rows (3), 8100 columns (6), n_lo 90 (3): GEMM tile 128x128
        # (pick 2 + tile 2); TTT FP32 with A and B k-fast, C's unit stride in
        # free A, M 7680 (6), N 120 (3), K 3072 (5): tile 256x32 (pick 6)
        tab.write_text("4 class:ttm|1|0|0|3|3|6|3\n6 class:ttt|1|1|1|1|6|3|5\n")
        T.autotune_load(str(tab))
        with Plan():
            for n in (90, 100):  # both shapes fall in the class
                A = _d((n, 90, n), _lib.F32)
                B = _d((64, 90), _lib.F32, ptr=FAKE * 2)
                C = _d((n, 64, n), _lib.F32, ptr=FAKE * 3)
                assert _ttm(A, B, 2, C) == 0
                p = _plan()
                assert "tile=128x128" in p and "autotuned(class)" in p, p
            Ad = _d((96, 80, 64, 48), _lib.F32, layout=(4, 3, 2, 1))
            Bd = _d((64, 48, 120), _lib.F32, ptr=FAKE * 2)
            Cd = _d((96, 80, 120), _lib.F32, ptr=FAKE * 3)
            L = _lib.lib()
            phi, psi = _lib.i32_array((1, 2, 3, 4)), _lib.i32_array((3, 1, 2))
            assert L.tlib_ttt(ctypes.byref(Ad), ctypes.byref(Bd), 2, phi, psi, ctypes.byref(Cd), None) == 0
            p = _plan()
            assert "tile=256x32" in p and "autotuned(class)" in p, p
            # a shape of another class takes the planner's rule
            A = _d((90, 90, 90), _lib.F32, layout=(3, 2, 1))
            B = _d((64, 90), _lib.F32, ptr=FAKE * 2)
            C = _d((64, 90, 90), _lib.F32, ptr=FAKE * 3, layout=(3, 2, 1))
            assert _ttm(A, B, 1, C) == 0
            assert "autotuned" not in _plan()
    finally:
        T.autotune_clear()
        T.set_autotune(prev)


def test_normalize_plan_and_errors():
    """tlib_normalize: a norm (dot kernel) then the division; shapes checked,
    in place allowed only on the very same view."""
    L = _lib.lib()
    with Plan():
        A = _d((7, 11, 13), _lib.F32)
        C = _d((7, 11, 13), _lib.BF16, ptr=FAKE * 2, layout=(3, 2, 1))
        nrm = ctypes.c_void_p(FAKE * 3)
        assert L.tlib_normalize(ctypes.byref(A), nrm, ctypes.byref(C), None) == 0
        p = _plan()
        assert "normalize dot" in p and "div dtype=f32->bf16 total=1001" in p, p
        assert L.tlib_normalize(ctypes.byref(A), nrm, ctypes.byref(A), None) == 0
        assert L.tlib_normalize(ctypes.byref(A), None, ctypes.byref(C), None) == _lib.EINVAL
        assert L.tlib_normalize(ctypes.byref(A), nrm, ctypes.byref(_d((7, 11, 12), _lib.F32, ptr=FAKE * 2)),
                                None) == _lib.ESHAPE
        A2 = _d((7, 11, 13), _lib.F32, layout=(2, 1, 3))  # same buffer, other strides
        assert L.tlib_normalize(ctypes.byref(A), nrm, ctypes.byref(A2), None) == _lib.EALIAS


def test_ttv_col_vector_width():
    """TTV col regime (Sec. 5.2 Eq. ttv): lanes along lo load the widest
    vector the strides allow, narrowed only while it would leave fewer than
    1024 workgroups; a k split then fills the chip."""
    L = _lib.lib()

    def plan(shape, q, dtype):
        A = _d(shape, dtype)
        b = _d((shape[q - 1],), dtype, ptr=FAKE * 2)
        C = _d(tuple(n for i, n in enumerate(shape) if i != q - 1), dtype, ptr=FAKE * 3)
        assert _ttv(A, b, q, C) == 0
        p = _plan()
        m = re.search(r"vec=(\d+) ksplit=(\d+) kr=\d+ blocks=(\d+)", p)
        assert "ttv col" in p and m, p
        return int(m.group(1)), int(m.group(2)), int(m.group(3))

    with Plan():
        # 406^3, mode 2: 16-byte vectors leave 4 x 406 = 1624 workgroups (>= 1024), split k in two
        assert plan((406, 406, 406), 2, _lib.F64) == (2, 2, 3248)
        assert plan((406, 406, 406), 2, _lib.F32)[0] == 2  # 4-wide: 812 < 1024, so 2-wide
        # 200 x 200 x 20: vectors would leave 40 workgroups, scalar loads leave 80; k split six ways
        assert plan((200, 200, 20), 2, _lib.F64) == (1, 6, 480)


def test_dot_partials_for_views():
    """Inner/norm partition (Sec. 5.2 Table 3 inner product and norm): a dense
    operand is one merged run split into a partial per 65536 elements (at most
    2048); a view whose dims do not merge goes by rows and takes at least one
    partial per 256 rows, up to 2048.  The workspace and the launch size their
    partials by the same rule."""
    L = _lib.lib()

    def partials(shape, strides, dtype=_lib.F32):
        A = _d(shape, dtype, strides=strides)
        out = ctypes.c_void_p(FAKE * 3)
        assert L.tlib_norm(ctypes.byref(A), out, None) == 0
        p = _plan()
        m = re.search(r"dims=(\d+) total=(\d+) partials=(\d+)", p)
        assert m, p
        return int(m.group(1)), int(m.group(2)), int(m.group(3))

    with Plan():
        # dense 90^4: one run, 65.6M elements -> ceil(65610000 / 65536) = 1002 partials
        assert partials((90, 90, 90, 90), None) == (1, 90 ** 4, 1002)
        # 90^4 window of a 100^4 parent: 729000 rows of 90 -> 2048 partials
        assert partials((90, 90, 90, 90), (1, 100, 100 ** 2, 100 ** 3)) == (4, 90 ** 4, 2048)
        # 1200 rows of 64: five partials (one per 256 rows), more than the two of the flat rule
        assert partials((64, 30, 40), (1, 70, 70 * 31)) == (3, 64 * 30 * 40, 5)
        # 100 rows of 10: one partial
        assert partials((10, 10, 10), (1, 12, 144)) == (3, 1000, 1)


def _tv(A, us, r, c):
    arr = (ctypes.POINTER(_lib.TensorDesc) * len(us))(
        *[ctypes.pointer(u) if u is not None else ctypes.POINTER(_lib.TensorDesc)() for u in us])
    return _lib.lib().tlib_times_vectors(ctypes.byref(A), arr, r, ctypes.byref(c), None)


def test_times_vectors_plans_and_errors():
    with Plan():
        n = 160
        A = _d((n,) * 4, _lib.F32)
        us = [_d((n,), _lib.F32, ptr=FAKE * (2 + k)) for k in range(4)]
        c = _d((n,), _lib.F32, ptr=FAKE * 9)
        # r = 1 is the stride-1 mode: its index runs over the tile positions
        assert _tv(A, us, 1, c) == 0 and _plan().startswith("times_vectors k1") and "vec=1" in _plan()
        # r = 4: one i_r per workgroup, every element of A read once
        assert _tv(A, us, 4, c) == 0 and _plan().startswith("times_vectors k2") and "out 25600 x hi 1" in _plan()
        # u_r is not read and may be NULL
        assert _tv(A, us[:1] + [None] + us[2:], 2, c) == 0
        # a view with gaps in the position modes takes the scalar path
        Ag = _d((n, n, n, n), _lib.F32, strides=(2, 2 * n, 2 * n * n, 2 * n ** 3))
        assert _tv(Ag, us, 2, c) == 0 and "vec=0" in _plan()
        # errors
        assert _tv(A, us, 0, c) == _lib.EMODE
        assert _tv(A, us, 5, c) == _lib.EMODE
        assert _tv(A, us[:2] + [_d((n + 1,), _lib.F32, ptr=FAKE * 4)] + us[3:], 1, c) == _lib.ESHAPE
        assert _tv(A, us, 1, _d((n + 1,), _lib.F32, ptr=FAKE * 9)) == _lib.ESHAPE
        assert _tv(A, us, 1, _d((n,), _lib.F64, ptr=FAKE * 9)) == _lib.EDTYPE
        assert _tv(A, us[:1] + [_d((n,), _lib.F64, ptr=FAKE * 3)] + us[2:], 1, c) == _lib.EDTYPE
        assert _tv(A, us, 1, _d((n,), _lib.F32, ptr=FAKE + 64)) == _lib.EALIAS
        assert _tv(_d((n,), _lib.F32), us[:1], 1, c) == _lib.EINVAL
        # 16-bit inputs give an FP32 result
        Ab = _d((n,) * 4, _lib.BF16)
        ub = [_d((n,), _lib.BF16, ptr=FAKE * (2 + k)) for k in range(4)]
        assert _tv(Ab, ub, 3, c) == 0


def test_ttm2_plans_and_errors():
    with Plan():
        n = 160
        L = _lib.lib()
        A = _d((n,) * 4, _lib.F32, layout=(4, 3, 2, 1))
        U = _d((32, n), _lib.F32, ptr=FAKE * 2)
        V = _d((32, n), _lib.F32, ptr=FAKE * 3)
        C = _d((32, 32, n, n), _lib.F32, layout=(4, 3, 2, 1), ptr=FAKE * 9)

        def call(A_, U_, a, V_, b, C_):
            return L.tlib_ttm2(ctypes.byref(A_), ctypes.byref(U_), a, ctypes.byref(V_), b, ctypes.byref(C_), None)

        assert call(A, U, 1, V, 2, C) == 0 and _plan().startswith("ttm2 fused") and "f=2 g=1" in _plan()
        # 40 factor rows: two TTMs through an intermediate
        U40 = _d((40, n), _lib.F32, ptr=FAKE * 2)
        C40 = _d((40, 32, n, n), _lib.F32, layout=(4, 3, 2, 1), ptr=FAKE * 9)
        assert call(A, U40, 1, V, 2, C40) == 0 and _plan().startswith("ttm2 chain")
        assert call(A, U, 1, V, 1, C) == _lib.EMODE
        assert call(A, U, 0, V, 2, C) == _lib.EMODE
        assert call(A, U, 1, V, 2, _d((32, 31, n, n), _lib.F32, ptr=FAKE * 9)) == _lib.ESHAPE
        assert call(A, _d((32, n + 1), _lib.F32, ptr=FAKE * 2), 1, V, 2, C) == _lib.ESHAPE
        Ab = _d((n,) * 4, _lib.BF16)
        Ub = _d((32, n), _lib.BF16, ptr=FAKE * 2)
        Vb = _d((32, n), _lib.BF16, ptr=FAKE * 3)
        assert call(Ab, Ub, 1, Vb, 2, C) == _lib.EDTYPE
        assert call(A, U, 1, V, 2, _d((32, 32, n, n), _lib.F32, ptr=FAKE + 64)) == _lib.EALIAS


def test_ewise_regimes():
    """Entrywise ops: the LDS-tiled relayout when C's fastest dim is not A's,
    the plain kernel otherwise; B read with A's tile or along C's lines."""
    L = _lib.lib()
    with Plan():
        A = _d((90, 90, 90), _lib.F32, layout=(3, 2, 1))
        Ad = _d((90, 90, 90), _lib.F32, ptr=FAKE * 4)
        C = _d((90, 90, 90), _lib.F32, ptr=FAKE * 2)
        B = _d((90, 90, 90), _lib.F32, layout=(3, 2, 1), ptr=FAKE * 3)
        assert L.tlib_scale(2.0, ctypes.byref(A), ctypes.byref(C), None) == 0
        assert _plan().startswith("scale ewise tile") and "x=90 y=90 rest=90 b=0" in _plan()
        assert L.tlib_add(1.0, ctypes.byref(A), 1.0, ctypes.byref(B), ctypes.byref(C), None) == 0
        assert "ewise tile" in _plan() and "b=2" in _plan()
        assert L.tlib_add(1.0, ctypes.byref(A), 1.0, ctypes.byref(Ad), ctypes.byref(C), None) == 0
        assert "ewise tile" in _plan() and "b=1" in _plan()
        # same layouts: one flat stream
        assert L.tlib_add(1.0, ctypes.byref(Ad), 1.0, ctypes.byref(Ad), ctypes.byref(C), None) == 0
        assert "ewise" in _plan() and "tile" not in _plan() and _plan().endswith("flat")
        # transpose of a matrix
        M = _d((300, 200), _lib.F64)
        Mt = _d((200, 300), _lib.F64, ptr=FAKE * 2)
        assert L.tlib_transpose(ctypes.byref(M), _lib.i32_array((2, 1)), ctypes.byref(Mt), None) == 0
        assert _plan().startswith("transpose ewise tile") and "x=200 y=300 rest=1" in _plan()
        # a short fastest dim (8 < 16) keeps the plain kernel
        S = _d((8, 500), _lib.F64, layout=(2, 1))
        Sc = _d((8, 500), _lib.F64, ptr=FAKE * 2)
        assert L.tlib_scale(1.0, ctypes.byref(S), ctypes.byref(Sc), None) == 0
        assert "tile" not in _plan()


def _req(op, A, B, mode, C, q=0, phi=None, psi=None):
    L = _lib.lib()
    pa = _lib.i32_array(phi) if phi is not None else None
    pb = _lib.i32_array(psi) if psi is not None else None
    return L.tlib_request_check(op, ctypes.byref(A) if A is not None else None,
                                ctypes.byref(B) if B is not None else None, mode, q, pa, pb,
                                ctypes.byref(C) if C is not None else None)


def test_request_check_rejects_before_reading():
    """A served request is validated in full before any descriptor field is
    copied: order beyond TLIB_MAX_ORDER, mode 0 or past the order, NULL
    extents, a non-permutation layout and unknown ops are refused with their
    codes, and a result the server places later (data NULL) is accepted."""
    A = _d((8, 9, 10))
    b = _d((9,), ptr=FAKE * 2)
    C = _lib.desc(0, _lib.F64, (8, 10))
    assert _req(0, A, b, 2, C) == _lib.OK
    big = _lib.desc(FAKE, _lib.F64, (2,) * 17)
    assert _req(0, big, b, 2, C) == _lib.EINVAL
    assert "order" in _lib.lib().tlib_last_error().decode()
    assert _req(0, A, b, 0, C) == _lib.EMODE
    assert _req(0, A, b, 4, C) == _lib.EMODE
    assert _req(1, A, _d((5, 9), ptr=FAKE * 2), 0, _lib.desc(0, _lib.F64, (8, 5, 10))) == _lib.EMODE
    noext = _lib.desc(FAKE, _lib.F64, (8, 9, 10))
    noext.extents = None
    assert _req(0, noext, b, 2, C) == _lib.EINVAL
    assert _req(0, _d((8, 9, 10), layout=(1, 1, 2)), b, 2, C) == _lib.EMODE
    assert _req(3, A, b, 2, C) == _lib.EINVAL
    assert _req(0, None, b, 2, C) == _lib.EINVAL
    # TTT: phi / psi must be given and be permutations
    B = _d((9, 10, 7), ptr=FAKE * 2)
    Ct = _lib.desc(0, _lib.F64, (8, 7))
    assert _req(2, A, B, 0, Ct, 2, (1, 2, 3), (3, 1, 2)) == _lib.OK
    assert _req(2, A, B, 0, Ct, 2, None, (3, 1, 2)) == _lib.EINVAL
    assert _req(2, A, B, 0, Ct, 2, (1, 2, 2), (3, 1, 2)) == _lib.EMODE
    assert _req(2, A, B, 0, Ct, 4, (1, 2, 3), (3, 1, 2)) == _lib.EINVAL


def test_config3_ttt_plans_split_k():
    """The (96,80,64,48) x (64,48,120) contraction has few output tiles, so it
    plans split-K partials (scratch from the stream's workspace)."""
    L = _lib.lib()
    with Plan():
        A = _d((96, 80, 64, 48), _lib.F32)
        B = _d((64, 48, 120), _lib.F32, ptr=FAKE * 2)
        C = _d((96, 80, 120), _lib.F32, ptr=FAKE * 3)
        rc = L.tlib_ttt(ctypes.byref(A), ctypes.byref(B), 2, _lib.i32_array((1, 2, 3, 4)),
                        _lib.i32_array((3, 1, 2)), ctypes.byref(C), None)
        assert rc == 0 and int(_plan().split("ksplit=")[1].split()[0]) > 1, _plan()


def _cache_stats():
    e, h, m = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _lib.lib().tlib_plan_cache_stats(ctypes.byref(e), ctypes.byref(h), ctypes.byref(m))
    return e.value, h.value, m.value


def test_plan_cache_reuses_plans():
    """A repeated call shape takes its plan from the cache (the plan text is
    the same and the hit count grows); another stride, mode or address
    alignment is a new shape (Sec. 3.1 Eq. stride.tuple.permutation: the
    strides decide the plan)."""
    L = _lib.lib()
    L.tlib_plan_cache_clear()
    phi, psi = _lib.i32_array((1, 2, 3, 4)), _lib.i32_array((3, 1, 2))
    calls = []
    for dt in (_lib.F64, _lib.F32):
        for lay in (None, (3, 2, 1), (2, 3, 1)):
            A = _d((40, 33, 29), dt, layout=lay)
            for m in (1, 2, 3):
                nb = [40, 33, 29]
                b = _d((nb[m - 1],), dt, ptr=FAKE * 2)
                cv = [n for i, n in enumerate(nb) if i != m - 1]
                C = _d(tuple(cv), _lib.F64 if dt == _lib.F64 else _lib.F32, ptr=FAKE * 3)
                calls.append(lambda A=A, b=b, m=m, C=C: _ttv(A, b, m, C))
                B = _d((17, nb[m - 1]), dt, ptr=FAKE * 2)
                cm = list(nb)
                cm[m - 1] = 17
                Cm = _d(tuple(cm), _lib.F64 if dt == _lib.F64 else _lib.F32, ptr=FAKE * 3)
                calls.append(lambda A=A, B=B, m=m, Cm=Cm: _ttm(A, B, m, Cm))
        At = _d((12, 10, 8, 6), dt, layout=(3, 1, 4, 2))
        Bt = _d((8, 6, 14), dt, ptr=FAKE * 2)
        Ct = _d((12, 10, 14), _lib.F64 if dt == _lib.F64 else _lib.F32, ptr=FAKE * 3)
        calls.append(lambda At=At, Bt=Bt, Ct=Ct: L.tlib_ttt(ctypes.byref(At), ctypes.byref(Bt), 2, phi, psi,
                                                           ctypes.byref(Ct), None))
    with Plan():
        first = []
        for f in calls:
            assert f() == 0
            first.append(_plan())
        e0, h0, m0 = _cache_stats()
        assert e0 == len(calls)
        for f, p0 in zip(calls, first):
            assert f() == 0
            assert _plan() == p0
        e1, h1, m1 = _cache_stats()
        assert (e1, h1 - h0, m1 - m0) == (e0, len(calls), 0)
        # the same TTV at an address 8 bytes off is another shape: FP64 lanes
        # along lo may no longer load 16-byte vectors
        A = _d((256, 4, 3000), _lib.F64, ptr=FAKE)
        A8 = _d((256, 4, 3000), _lib.F64, ptr=FAKE + 8)
        b = _d((4,), _lib.F64, ptr=FAKE * 2)
        C = _d((256, 3000), _lib.F64, ptr=FAKE * 3)
        assert _ttv(A, b, 2, C) == 0
        p_al = _plan()
        assert _ttv(A8, b, 2, C) == 0
        p_un = _plan()
        assert "vec=2" in p_al and "vec=1" in p_un, (p_al, p_un)
        assert _cache_stats()[0] == e0 + 2
    L.tlib_plan_cache_clear()
    assert _cache_stats()[0] == 0


def test_grouped_launch_rejects_long_contractions():
    """A grouped thread or tile carries a request's whole contraction in one
    accumulator chain, so requests with a contraction above TLIB_BATCH_MAX_K
    (8192) are not groupable; the single entry points split them.  TTV with
    n_m = 8192 / 8193 and TTT contracting every mode of A (K = 8192 / 9000)."""
    L = _lib.lib()

    def req(op, A, B, C, mode=0, q=0, phi=None, psi=None):
        r = _lib.Request()
        r.op, r.mode, r.q = op, mode, q
        r.A, r.B, r.C = ctypes.pointer(A), ctypes.pointer(B), ctypes.pointer(C)
        keep = []
        if phi is not None:
            pa, pb = _lib.i32_array(phi), _lib.i32_array(psi)
            keep += [pa, pb]
            r.phi = ctypes.cast(pa, ctypes.POINTER(ctypes.c_int32))
            r.psi = ctypes.cast(pb, ctypes.POINTER(ctypes.c_int32))
        return r, keep

    for nk, want in ((8192, 1), (8193, 0)):
        A = _d((nk, 3), _lib.F32)
        b = _d((nk,), _lib.F32, ptr=FAKE * 2)
        C = _d((3,), _lib.F32, ptr=FAKE * 3)
        r, keep = req(0, A, b, C, mode=1)
        assert L.tlib_request_groupable(ctypes.byref(r)) == want, nk
    for shape, want in (((64, 128), 1), ((90, 100), 0)):
        A = _d(shape, _lib.F32)
        B = _d(shape + (8,), _lib.F32, ptr=FAKE * 2)
        C = _d((8,), _lib.F32, ptr=FAKE * 3)
        r, keep = req(2, A, B, C, q=2, phi=(1, 2), psi=(3, 1, 2))
        assert L.tlib_request_groupable(ctypes.byref(r)) == want, shape
    # the batch planner rejects the long one with TLIB_EINVAL and names it
    arr = (_lib.Request * 1)(r)
    nbytes = L.tlib_batch_table_bytes(1)
    host = (ctypes.c_char * nbytes)()
    units, bad = ctypes.c_int64(0), ctypes.c_int32(-1)
    assert L.tlib_batch_plan(arr, 1, host, nbytes, ctypes.byref(units), ctypes.byref(bad)) == _lib.EINVAL
    assert bad.value == 0 and b"8192" in L.tlib_last_error()
