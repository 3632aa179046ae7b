"""GPU parity of the tensor-grid preview (fst_eval_grid, Sec. 6 fast visualisation) through
the C ABI, against the oracle's mode-product form (itself pinned against eq. (1) point by
point) and against the GPU's own point-by-point reconstruction.

Tolerances (relative L2 over the grid): FP64 1e-10, FP32 1e-5.  FP32 coordinates are given
to the oracle as the same float32 numbers up-cast exactly, so the comparison measures kernel
arithmetic only.
"""
import ctypes as C

import numpy as np
import pytest

import datagen
from oracle import reconstruct
from oracle.model import Model as OModel
from oracle.reconstruct import rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
fst = pytest.importorskip("paper_1907_05884_amd.binding")

LO, HI = (0.0, -2.0, 1.0), (4.0, 1.0, 3.0)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def D(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def H(t):
    return t.detach().cpu().numpy()


def _models(seed, rank, degree):
    core, coefs = datagen.random_model_parts(seed, rank, degree)
    om = OModel(LO, HI, tuple(rank), tuple(degree), core, coefs)
    gm = fst.fst_model_from_parts(LO, HI, rank, degree, core, coefs)
    return om, gm


def _axes(seed, shape, dtype):
    rng = np.random.default_rng(seed)
    return [rng.uniform(LO[k], HI[k], shape[k]).astype(dtype) for k in range(3)]


# shapes: ragged counts (not multiples of the 256-column or 32-row blocks), 2-D slices along
# each axis, a single point; ranks: not multiples of 8 (padded contraction), and the maximum.
# FP32 column counts that are multiples of 4 take the four-column (16-byte store) path of the
# mode products: (45, 12, 68) has 68 and 816 columns, ragged against its 1024-column blocks
@pytest.mark.parametrize("dtype,rank,degree,shape,tol", [
    (np.float64, (7, 12, 5), (9, 14, 6), (37, 1, 53), 1e-10),
    (np.float64, (32, 32, 32), (31, 31, 31), (64, 65, 33), 1e-10),
    (np.float64, (3, 4, 2), (5, 4, 6), (1, 1, 1), 1e-10),
    (np.float64, (16, 1, 9), (20, 3, 11), (300, 2, 1), 1e-10),
    (np.float32, (24, 24, 24), (31, 31, 31), (130, 70, 257), 1e-5),
    (np.float32, (9, 17, 31), (12, 20, 31), (1, 300, 299), 1e-5),
    (np.float32, (5, 11, 24), (8, 15, 29), (45, 12, 68), 1e-5),
])
def test_grid_matches_oracle(dev, dtype, rank, degree, shape, tol):
    print(f"grid {shape} rank {rank} {np.dtype(dtype).name}", flush=True)
    om, gm = _models(sum(rank), rank, degree)
    g = _axes(sum(shape), shape, dtype)
    ref = reconstruct.evaluate_tensor_grid(om, *[a.astype(np.float64) for a in g])
    out = fst.fst_eval_grid(gm, *[D(a, dev) for a in g])
    assert tuple(out.shape) == shape and out.dtype == D(g[0], dev).dtype
    assert rel_l2(H(out), ref) <= tol


def test_large_grid_against_pointwise_and_sampled_oracle(dev):
    # 256^3 FP32 grid of a rank-24^3 model: the whole grid against the GPU's point-by-point
    # reconstruction (eq. (1) per point, 2R flop each), and 2000 sampled grid points against
    # the oracle
    shape = (256, 256, 256)
    print(f"grid {shape} rank 24^3 float32", flush=True)
    om, gm = _models(11, (24, 24, 24), (31, 31, 31))
    g = _axes(5, shape, np.float32)
    gd = [D(a, dev) for a in g]
    out = fst.fst_eval_grid(gm, *gd)
    X, Y, Z = torch.meshgrid(*gd, indexing="ij")
    pw = fst.fst_eval(gm, X.contiguous().view(-1), Y.contiguous().view(-1), Z.contiguous().view(-1))
    assert rel_l2(H(out).reshape(-1), H(pw)) <= 1e-5
    rng = np.random.default_rng(3)
    ii = [rng.integers(0, s, 2000) for s in shape]
    P = np.stack([g[k][ii[k]].astype(np.float64) for k in range(3)], axis=1)
    ref = reconstruct.evaluate(om, P)
    got = H(out)[ii[0], ii[1], ii[2]]
    assert rel_l2(got, ref) <= 1e-5


def test_grid_without_workspace_and_bad_counts(dev):
    om, gm = _models(2, (5, 6, 7), (8, 8, 8))
    g = _axes(9, (20, 21, 22), np.float64)
    gd = [D(a, dev) for a in g]
    out = torch.empty((20, 21, 22), dtype=torch.float64, device=dev)
    st = fst._fn["fst_eval_grid"](gm.handle, fst.FST_F64, gd[0].data_ptr(), 20, gd[1].data_ptr(), 21,
                                  gd[2].data_ptr(), 22, out.data_ptr(), None, 0,
                                  C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == fst.FST_OK
    ref = reconstruct.evaluate_tensor_grid(om, *g)
    assert rel_l2(H(out), ref) <= 1e-10
    with pytest.raises(fst.FstError) as e:
        fst.fst_eval_grid(gm, gd[0][:0], gd[1], gd[2])
    assert e.value.status == fst.FST_E_INVAL
