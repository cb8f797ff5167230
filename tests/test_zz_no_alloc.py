"""tdb_reconstruct_noalloc (for callers that cannot allocate device memory) against
the existing tdb_reconstruct of a handle holding the same factors: two calls in a
row, the second on a smaller tensor, in FP64 (bar 1e-12 relative: the same FP64
products, possibly summed in another order) and FP32 data (bar 1e-6: the handle's
chain runs in FP32, this one in FP64 rounded once)."""
import ctypes
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BAR = {"f64": 1e-12, "f32": 1e-6}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2201_06958_amd import load_library
    load_library()


def _factors(rng, dims, ranks):
    C = rng.normal(size=ranks)
    U = []
    for n, r in zip(dims, ranks):
        q, _ = np.linalg.qr(rng.normal(size=(n, r)))
        U.append(q * np.sqrt(n))           # W-orthonormal for the default weights 1/N
    return C, U


def _reference(dims, ranks, C, U, dtype):
    from paper_2201_06958_amd import Compressor
    V0 = torch.zeros(dims, dtype=torch.float32 if dtype == "f32" else torch.float64, device="cuda")
    g = Compressor(dims, 0.01, rank_max=ranks, rank_init=ranks, data_dtype=dtype,
                   precision="f32" if dtype == "f32" else "f64", adaptive=False, eps_th=1.0, path="plain")
    g.init_from_factors(V0, C, U)
    out = g.reconstruct().cpu().numpy()
    g.close()
    return out


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_matches_reconstruct_two_calls(dtype):
    from paper_2201_06958_amd.tdb import reconstruct_noalloc
    rng = np.random.default_rng(21)
    cases = [((40, 36, 12), (6, 5, 4)), ((20, 18, 6), (3, 3, 2))]   # the second call is smaller
    for dims, ranks in cases:
        _say(f"case noalloc {dtype} dims {dims} ranks {ranks}")
        C, U = _factors(rng, dims, ranks)
        ref = _reference(dims, ranks, C, U, dtype)
        Cd = torch.from_numpy(C).cuda()
        Ud = [torch.from_numpy(np.ascontiguousarray(u)).cuda() for u in U]
        out = torch.empty(dims, dtype=torch.float32 if dtype == "f32" else torch.float64, device="cuda")
        reconstruct_noalloc(Cd, Ud, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        rel = float(np.abs(got.astype(np.float64) - ref).max() / np.abs(ref).max())
        _say(f"  rel diff to tdb_reconstruct {rel:.2e}")
        assert rel < BAR[dtype]


def test_noalloc_fourth_order_and_scratch_limit():
    from paper_2201_06958_amd import tdb
    from paper_2201_06958_amd.tdb import TDBError, reconstruct_noalloc
    rng = np.random.default_rng(5)
    dims, ranks = (14, 12, 10, 3), (4, 3, 3, 2)
    _say(f"case noalloc order 4 dims {dims}")
    C, U = _factors(rng, dims, ranks)
    ref = _reference(dims, ranks, C, U, "f64")
    out = torch.empty(dims, dtype=torch.float64, device="cuda")
    reconstruct_noalloc(torch.from_numpy(C).cuda(), [torch.from_numpy(np.ascontiguousarray(u)).cuda() for u in U],
                        out)
    torch.cuda.synchronize()
    assert float(np.abs(out.cpu().numpy() - ref).max() / np.abs(ref).max()) < 1e-12
    # an intermediate above half the scratch (here 2048 x 2048 x 4 doubles after the
    # first product) is refused before any launch (the small buffers are never read)
    big = (2048, 2048, 4)
    Cb = torch.zeros((1, 1, 1), dtype=torch.float64, device="cuda")
    Ub = [torch.zeros((1, 1), dtype=torch.float64, device="cuda") for _ in big]
    ob = torch.empty((1,), dtype=torch.float64, device="cuda")
    lib = tdb.load_library()
    dims_c = (ctypes.c_int64 * 8)(*big, 0, 0, 0, 0, 0)
    ranks_c = (ctypes.c_int32 * 8)(*big, 0, 0, 0, 0, 0)
    uptr = (ctypes.c_void_p * 8)(*[u.data_ptr() for u in Ub], None, None, None, None, None)
    st = lib.tdb_reconstruct_noalloc(3, dims_c, ranks_c, ctypes.c_void_p(Cb.data_ptr()), uptr, tdb.F64,
                                     ctypes.c_void_p(ob.data_ptr()), None)
    assert st == tdb.EINVAL
    assert b"scratch" in lib.tdb_last_error(None)
