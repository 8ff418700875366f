"""GPU parity of the sliced-ELLPACK (SELL-C-sigma) handles: element by element
against the oracle, and bit for bit against CSR handles of the same matrix
(both add the rounded products of a row in ascending order), in every
precision, for several sigma, with empty rows, long rows and NaN/Inf in x."""
import numpy as np
import pytest
import torch

import meshgen as mg
import oracle
import paper_2107_12371_amd as spmv

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
SELL = {"format": spmv.FORMAT_SELL}


def to_dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype)


def products(A, x, params, **kw):
    with spmv.Matrix.from_csr(A, fp32=True, bf16=True, params=params, **kw) as M:
        xd = to_dev(x)
        out = {"f64": M.apply(xd).cpu().numpy(), "f32": M.apply_f32(xd.float()).cpu().numpy(),
               "f32v": M.apply_f32v(xd).cpu().numpy(), "bf16": M.apply_bf16(xd.float()).cpu().numpy(),
               "info": M.info}
    return out


CASES = {
    "mesh32": lambda: mg.config0(),
    "edge_long_empty": lambda: mg.random_csr(5000, 3000, seed=21, mean_len=5.0, empty_frac=0.3, dense_rows=4),
    "duplicates_unsorted": lambda: mg.random_csr(4099, 777, seed=22, mean_len=9.0, duplicates=True,
                                                 unsorted=True),
    "knn_random_order": lambda: mg.config1("random", m=40),
}


@pytest.mark.parametrize("name", list(CASES))
def test_sell_matches_oracle_and_csr_bitwise(name):
    A = CASES[name]()
    x = mg.uniform(A.n_cols, 31, 0)
    s = products(A, x, SELL)
    c = products(A, x, {"window_mode": spmv.WINDOW_OFF})
    assert s["info"]["format"] == spmv.FORMAT_SELL and s["info"]["n_slices"] == (
        int(np.sum(np.diff(A.row_ptr) <= 255)) + 63) // 64
    y_ref, bound = oracle.spmv(A, x)
    assert oracle.spmv_accept(s["f64"], y_ref, bound).all()
    for k in ("f64", "f32", "f32v", "bf16"):
        assert np.array_equal(s[k], c[k]), k


def test_sell_sigma_and_xcd_order_do_not_change_bits():
    A = mg.config1("rcm", m=50)
    x = mg.uniform(A.n_cols, 32, 0)
    ref = products(A, x, SELL)["f64"]
    for sigma in (64, 512, 32768):
        assert np.array_equal(products(A, x, {"format": spmv.FORMAT_SELL, "sell_sigma": sigma})["f64"], ref)
    assert np.array_equal(products(A, x, SELL, xcd_remap=False)["f64"], ref)


def test_sell_dyadic_bitwise_and_nonfinite():
    A = mg.config0(dyadic=True)
    x = mg.dyadic_x(A.n_cols, seed=5)
    y = products(A, x, SELL)["f64"]
    assert np.array_equal(y, oracle.spmv(A, x)[0])
    B = mg.random_csr(600, 600, seed=23, mean_len=6.0, empty_frac=0.1)
    xb = mg.uniform(B.n_cols, 33, 0)
    xb[[4, 90]] = np.nan
    xb[[17]] = -np.inf
    yb = products(B, xb, SELL)["f64"]
    y_ref, bound = oracle.spmv(B, xb)
    assert np.isnan(y_ref).any() and oracle.spmv_accept(yb, y_ref, bound).all()


@pytest.mark.parametrize("mode", [spmv.CG_FP64, spmv.CG_MIXED_FP32])
def test_sell_cg(mode):
    A = mg.config0()
    b = mg.uniform(A.n_rows, 34, 4)
    with spmv.Matrix.from_csr(A, fp32=True, params=SELL) as M:
        x, info = M.cg(to_dev(b), tol=1e-10, mode=mode)
        x = x.cpu().numpy()
    Ax, _ = oracle.spmv(A, x)
    assert np.linalg.norm(b - Ax) / np.linalg.norm(b) <= 1.05e-10
    assert info.iterations > 0


def test_sell_empty_and_bad_format():
    A = mg.CSR(4, 3, np.zeros(5, np.int32), np.zeros(0, np.int32), np.zeros(0))
    with spmv.Matrix.from_csr(A, params=SELL) as M:
        assert np.all(M.apply(to_dev(np.ones(3))).cpu().numpy() == 0.0)
    with pytest.raises(spmv.SpmvError) as e:
        spmv.Matrix.from_csr(mg.config0(), params={"format": 7})
    assert e.value.code == spmv.SPMV_EINVAL
