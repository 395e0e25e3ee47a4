"""GPU parity of the DGETT emulated on INT8 MFMA (Ozaki scheme, dgett_ozaki).

Bars: with one K slice (K <= 16384) the GPU follows the oracle's model step
for step -- the same exponents and slices, exact integer slice-pair sums,
the same double combination and C_in + v -- so GPU == C_in + model bit for
bit, whatever the data; with several K slices each slice's value is combined
on its own and C <- C_in + v_1 + v_2 + ... in slice order, within
(2S + 4) u64 sum|a||b| of the model; integer inputs are
exact; against the exact result, e_nrm <= 1e-12 with 8 slices on normal(0,1)
data, and the scheme's own bound K 2^(eA+eB) (S+1) 2^-7S holds for fewer.
C-parent elements outside C's view keep their sentinel.
"""
import zlib

import numpy as np
import pytest

import oracle
from paper_2410_06770_amd import gett, workloads as W
from tests.helpers import call14, e_nrm, outside_mask, to_device, view_values

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53


@pytest.fixture(scope="module", autouse=True)
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gett.lib()
    gett.use_torch_stream()
    yield
    torch.cuda.synchronize()


def run(pr, slices, tag=""):
    import torch
    print(f"\n[gpu] ozaki S={slices} {tag} {pr.name} sig={pr.signature()}", flush=True)
    At, a = to_device(pr.A)
    Bt, b = to_device(pr.B)
    Ct, c = to_device(pr.C)
    rc = call14(lambda *args: gett.dgett_ozaki(*args, slices=slices), pr, a, b, c)
    assert rc == 0, gett.strerror(rc)
    torch.cuda.synchronize()
    return Ct.cpu().numpy()


def row_index(pr):
    """(ra, rb): for every output of C's view, in view order, the canonical
    row of A and of B it is the product of."""
    fa, fb = pr.free_modes()
    extc = pr.extc()
    grid = np.indices(extc)
    ra = np.zeros(extc, dtype=np.int64)
    rb = np.zeros(extc, dtype=np.int64)
    s = 1
    for p, i in enumerate(fa):
        ra = ra + grid[pr.perm[p]] * s
        s *= pr.exta[i]
    s = 1
    for p, j in enumerate(fb):
        rb = rb + grid[pr.perm[len(fa) + p]] * s
        s *= pr.extb[j]
    return ra, rb


def model_and_exponents(pr, slices):
    """The oracle's Ozaki model v (no C_in) at C's view, view order, with the
    row exponents it used and K."""
    rA, rB, kA, kB = oracle.canonical_offsets(pr)
    QA, EA = oracle.ozaki_split(pr.A, rA, kA, slices)
    QB, EB = oracle.ozaki_split(pr.B, rB, kB, slices)
    model = oracle.ozaki_gemm(QA, EA, QB, EB, len(kA), slices)
    if not pr.extc():
        return model.reshape(()), EA, EB, len(kA)
    ra, rb = row_index(pr)
    return model[ra, rb], EA, EB, len(kA)


def check_model(pr, got, slices, tol=0.0):
    """GPU == C_in + model bit for bit (tol 0), else within tol of sum|a||b|."""
    m, _, _, _ = model_and_exponents(pr, slices)
    exp = view_values(pr.C) + m
    cv = view_values(pr.C, got)
    if tol == 0.0:
        assert np.array_equal(cv, exp), int(np.sum(cv != exp))
    else:
        _, cabs = oracle.exact(pr, pr.A, pr.B, pr.C)
        assert np.all(np.abs(cv - exp) <= tol * view_values(pr.C, cabs))
    mask = outside_mask(pr.C)
    assert np.array_equal(got[mask], pr.C.buf[mask])


@pytest.mark.parametrize("case", W.PAPER_CASES)
def test_paper_families_follow_the_model_bitwise(case):
    rng = np.random.default_rng(zlib.crc32(case.encode()) + 900)
    for S in (8, 5):
        for dist in ("normal", "int"):
            pr = W.paper_case(case, rng, dtype=np.float64, dist=dist)
            got = run(pr, S, f"{case} {dist}")
            check_model(pr, got, S)


@pytest.mark.parametrize("slices", [3, 4, 5, 6, 7, 8])
def test_every_slice_count_on_a_strided_problem(slices):
    """Strided + permuted, both loader shapes (A's rows along its fastest
    mode, B's contracted positions along its), ragged M and N, K spanning
    more than one 512-position group."""
    rng = np.random.default_rng(920 + slices)
    sig = (4, [13, 17, 30, 25], 4, [25, 11, 30, 9], 2, [2, 3], [2, 0], [2, 0, 3, 1])
    pr = W.build_problem(rng, sig, np.float64, "step2", "packed", "sub", dist="normal")
    A_vals = pr.A.buf[pr.A.element_index()]
    pr.A.buf[pr.A.element_index()] = A_vals * 2.0 ** rng.integers(-30, 30, A_vals.size)
    got = run(pr, slices, "strided")
    check_model(pr, got, slices)


def test_integer_inputs_are_exact():
    rng = np.random.default_rng(930)
    sig = (3, [70, 40, 33], 3, [33, 50, 40], 2, [1, 2], [2, 0], [0, 1])
    pr = W.build_problem(rng, sig, np.float64, "sub", "neg", "sub", dist="int")
    got = run(pr, 3, "int")
    ref, _ = oracle.exact(pr, pr.A, pr.B, pr.C)
    sel = ~np.isnan(ref)
    assert np.array_equal(got[sel], ref[sel])


def test_several_k_slices():
    """K = 20000 (over the 16384 positions one INT32 sum takes): the K slices'
    values are added to C_in in slice order, within (2S + 4) u64 sum|a||b| of
    the model, and the result stays within e_nrm 1e-12 of the exact one."""
    rng = np.random.default_rng(940)
    sig = (2, [20000, 37], 2, [20000, 29], 1, [0], [0], [0, 1])
    pr = W.build_problem(rng, sig, np.float64, "packed", "packed", "sub", dist="normal")
    got = run(pr, 8, "two K slices")
    check_model(pr, got, 8, tol=20 * U64)
    ref, _ = oracle.exact(pr, pr.A, pr.B, pr.C)
    sel = ~np.isnan(ref)
    assert e_nrm(got[sel], ref[sel]) <= 1e-12


@pytest.mark.parametrize("slices", [3, 4])
def test_error_within_the_scheme_bound(slices):
    rng = np.random.default_rng(950 + slices)
    sig = (2, [60, 300], 2, [300, 45], 1, [1], [0], [0, 1])
    pr = W.build_problem(rng, sig, np.float64, "packed", "packed", "sub", dist="normal")
    got = run(pr, slices, "bound")
    ref, cabs = oracle.exact(pr, pr.A, pr.B, pr.C)
    _, EA, EB, K = model_and_exponents(pr, slices)
    ra, rb = row_index(pr)
    bnd = K * 2.0 ** (EA[ra] + EB[rb]).astype(np.float64) * (slices + 1) * 2.0 ** (-7 * slices)
    err = np.abs(view_values(pr.C, got) - view_values(pr.C, ref))
    assert np.all(err <= bnd + 4 * U64 * view_values(pr.C, cabs))
    assert err.max() > 1e-3 * bnd.max()


def test_strided_workload_full_size_sampled():
    """The strided + permuted FP64 workload at full size, 8 slices: e_nrm
    against the exact values at 4000 outputs."""
    pr = W.config_strided_perm(dtype=np.float64)
    got = run(pr, 8, "full size")
    ref, _ = oracle.exact(pr, pr.A, pr.B, pr.C, 0, 4000)
    sel = ~np.isnan(ref)
    en = e_nrm(got[sel], ref[sel])
    print(f"[ozaki] strided e_nrm {en:.3e}", flush=True)
    assert en <= 1e-12
