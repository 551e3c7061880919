"""stkfmm_direct_noalloc: the FP64 direct sum with its per-slice partial sums
in the library's static device scratch instead of allocated memory.  It uses
the same source slices as stkfmm_direct, so its results must equal
stkfmm_direct's bit for bit, call after call (the scratch keeps the previous
call's contents), and sizes whose partial sums exceed the scratch are
refused before any launch."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2010_15155_amd import FMM, StkfmmError, kernel_dims, workloads as W

pytestmark = pytest.mark.gpu


def _inputs(kernel, n_src, n_trg, seed):
    rng = np.random.default_rng(seed)
    k_sl, k_dl, _ = kernel_dims(kernel)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    y = dev(rng.random((n_src, 3)))
    v = dev(rng.standard_normal((n_src, k_sl)))
    if kernel == "RPY":
        v[:, 3] = torch.from_numpy(rng.uniform(0.002, 0.005, n_src)).cuda()
    dl = dlv = None
    if k_dl:
        dl = dev(rng.random((n_src // 2, 3)))
        dlv = dev(rng.standard_normal((n_src // 2, k_dl)))
    x = dev(rng.random((n_trg, 3)))
    return y, v, dl, dlv, x


@pytest.mark.parametrize("kernel", ["Stokeslet", "RPY", "PVel", "Traction"])
def test_noalloc_matches_direct_twice(kernel):
    print("no-alloc direct: %s, 3000 then 1000 targets" % kernel, flush=True)
    fmm = FMM()
    try:
        for n_src, n_trg, seed in ((20000, 3000, 1), (8000, 1000, 2)):
            y, v, dl, dlv, x = _inputs(kernel, n_src, n_trg, seed)
            ref = fmm.direct(kernel, y, v, dl, dlv, x)
            out = torch.full_like(ref, float("nan"))
            got = fmm.direct(kernel, y, v, dl, dlv, x, out=out, noalloc=True)
            torch.cuda.synchronize()
            assert got.data_ptr() == out.data_ptr()
            assert torch.isfinite(got).all()
            # identical slices and summation order: bit-for-bit equal
            assert torch.equal(got, ref), float((got - ref).abs().max())
    finally:
        fmm.close()


def test_noalloc_matches_direct_large_target_count():
    # above about 5e5 targets the sum is not sliced and needs no scratch
    print("no-alloc direct: Stokeslet, 600000 targets, 2000 sources", flush=True)
    fmm = FMM()
    try:
        y, v, _, _, x = _inputs("Stokeslet", 2000, 600000, 3)
        ref = fmm.direct("Stokeslet", y, v, None, None, x)
        got = fmm.direct("Stokeslet", y, v, None, None, x, noalloc=True)
        assert torch.equal(got, ref)
    finally:
        fmm.close()


def test_noalloc_refuses_sizes_beyond_scratch():
    # PVelGrad (16 values per target): 2304 targets over 233472 sources are
    # split into 228 slices, 228 * 2304 * 16 doubles > 2^23
    print("no-alloc direct: PVelGrad beyond the scratch (refused on the host)", flush=True)
    fmm = FMM()
    try:
        y, v, _, _, x = _inputs("PVelGrad", 233472, 2304, 4)
        with pytest.raises(StkfmmError) as e:
            fmm.direct("PVelGrad", y, v, None, None, x, noalloc=True)
        assert e.value.status == "E_ARG" and "static scratch" in str(e.value)
        # the context stays usable, and below the limit the call succeeds
        ref = fmm.direct("PVelGrad", y[:5000], v[:5000], None, None, x)
        got = fmm.direct("PVelGrad", y[:5000], v[:5000], None, None, x, noalloc=True)
        assert torch.equal(got, ref)
    finally:
        fmm.close()
