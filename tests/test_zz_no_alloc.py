"""The no-allocation entry point (qa_integrate_noalloc) against qa_integrate:
same set, tile and grid, one round each, two calls in a row (the second with
a smaller input, so that stale contents of the library's scratch array would
show): the accumulator records must be bit-identical."""
import ctypes as C

import numpy as np
import pytest

import paper_1905_08007_amd as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _noalloc(s, img, budgets, seed, tag, tile, grid, acc):
    b = np.ascontiguousarray(budgets, dtype=np.uint64)
    L = P.lib()
    f = L.qa_integrate_noalloc
    f.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                  C.c_void_p, C.c_void_p]
    rc = f(s.h, img.ptr, b.ctypes.data_as(C.c_void_p), 0, seed, tag, tile, grid, C.c_void_p(acc.data_ptr()),
           C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, L.qa_last_error()


@pytest.mark.parametrize("loops,first_b,second_b", [
    (2, [100_003, 64, 70_001, 1], [5_000, 0, 300, 7]),
    (3, [4_096 + 17 * i for i in range(28)], [257 if i % 3 else 0 for i in range(28)]),
])
def test_noalloc_matches_integrate(loops, first_b, second_b):
    gs = P.enumerate_graphs(loops)
    s = P.build_forests(gs)
    p = P.pdf_create(s)
    img = P.upload(s, p)
    tile, grid = 256, 1024
    for budgets, seed in ((first_b, 11), (second_b, 12)):
        ref = P.read_acc(P.integrate(s, img, budgets, seed=seed, tag=0, tile=tile, grid=grid))
        acc = torch.full((len(gs) * P.ACC_BYTES,), 0xAB, dtype=torch.uint8, device="cuda")   # not zero: must be cleared
        _noalloc(s, img, budgets, seed, 0, tile, grid, acc)
        torch.cuda.synchronize()
        got = P.read_acc(acc)
        assert got.tobytes() == ref.tobytes(), (loops, budgets)
        assert [int(x["n"]) + int(x["n_bad"]) for x in got] == list(budgets)


def test_noalloc_rejects_bad_arguments():
    gs = P.enumerate_graphs(2)
    s = P.build_forests(gs)
    p = P.pdf_create(s)
    img = P.upload(s, p)
    acc = P.new_acc(len(gs))
    L = P.lib()
    L.qa_integrate_noalloc.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.c_uint64, C.c_uint32,
                                       C.c_uint32, C.c_uint32, C.c_void_p, C.c_void_p]
    b = np.array([64] * 4, dtype=np.uint64)
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.qa_integrate_noalloc(s.h, img.ptr, b.ctypes.data_as(C.c_void_p), 0, 1 << 32, 0, 256, 0,
                                  C.c_void_p(acc.data_ptr()), st) != 0
    assert L.qa_integrate_noalloc(s.h, img.ptr, b.ctypes.data_as(C.c_void_p), 0, 1, 0, 100, 0,
                                  C.c_void_p(acc.data_ptr()), st) != 0
