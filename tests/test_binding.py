"""The Python binding's argument marshalling for the batched calls (host
arrays handed to the C ABI).  CPU only."""
import ctypes

import numpy as np
import pytest

import paper_1908_09606_amd as cm


def test_int64_arrays():
    a = cm._i64arr([1, 2, np.int64(3), 4.0, 2**40])
    assert isinstance(a, ctypes.Array) and a._type_ is ctypes.c_int64
    assert list(a) == [1, 2, 3, 4, 2**40]
    assert list(cm._i64arr(x for x in (5, 6))) == [5, 6]
    assert list(cm._i64arr(np.arange(4))) == [0, 1, 2, 3]
    assert len(cm._i64arr([])) == 0


def test_double_arrays():
    d = cm._dblarr([1, 2.5, np.float64(-3.25), np.float32(0.5)])
    assert d._type_ is ctypes.c_double
    assert list(d) == [1.0, 2.5, -3.25, 0.5]
    assert list(cm._dblarr(iter([0.125]))) == [0.125]


def test_pointer_arrays():
    torch = pytest.importorskip("torch")
    t = torch.empty(7)
    p = cm._ptrarr([t, t])
    assert p._type_ is ctypes.c_void_p
    assert [x for x in p] == [t.data_ptr(), t.data_ptr()]
    # integers and None (a null pointer) go through the generic path
    q = cm._ptrarr([None, 4096, t])
    assert q[0] is None and q[1] == 4096 and q[2] == t.data_ptr()
    assert [x for x in cm._ptrarr(iter([t]))] == [t.data_ptr()]
    with pytest.raises(TypeError):
        cm._ptrarr([object()])


def test_arrays_outlive_their_sources():
    # the ctypes array must keep its buffer alive after the input is gone
    a = cm._i64arr(list(range(1000)))
    junk = [list(range(1000)) for _ in range(50)]
    assert list(a)[:3] == [0, 1, 2] and a[999] == 999
    del junk


def test_batched_size_query_same_for_lists_and_arrays():
    m, n, k = [100, 300, 64], [200, 50, 64], [1000, 70, 4096]
    rc1, b1 = cm.cosma_workspace_size_batched(3, m, n, k, [1.0] * 3, cm.COSMA_F32)
    rc2, b2 = cm.cosma_workspace_size_batched(3, np.array(m), np.array(n), np.array(k),
                                              np.ones(3), cm.COSMA_F32)
    assert rc1 == rc2 == 0 and b1 == b2 > 0
