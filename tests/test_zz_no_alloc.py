"""The allocation-free entry point ccsd_k_zgemm_noalloc (for callers that cannot allocate
device memory) against the allocating ccsd_k_debug_zgemm, through the C ABI: same kernels,
so the outputs agree bit for bit; two calls in a row on the shared scratch array, the
second with smaller sizes (its tables overwrite the first call's)."""
import numpy as np
import pytest

ck = pytest.importorskip("paper_1911_00242_amd", reason="libccsdk.so not built")
torch = pytest.importorskip("torch")


def test_noalloc_rejects_bad_and_too_large_sizes():
    """Argument checks that run before any device work (host only)."""
    fake = 1 << 20  # never dereferenced: the call is refused first
    with pytest.raises(ck.CcsdKError) as e:
        ck.ccsd_k_zgemm_noalloc(1, 4096, 4096, 4096, fake, fake, fake, 2)
    assert e.value.code == ck.EINVAL and "scratch" in ck.ccsd_k_last_error(None)
    with pytest.raises(ck.CcsdKError) as e:
        ck.ccsd_k_zgemm_noalloc(1, 8, 8, 8, fake, fake, fake, 5)
    assert e.value.code == ck.EINVAL
    with pytest.raises(ck.CcsdKError) as e:
        ck.ccsd_k_zgemm_noalloc(0, 8, 8, 8, fake, fake, fake, 0)
    assert e.value.code == ck.EINVAL
    with pytest.raises(ck.CcsdKError) as e:
        ck.ccsd_k_zgemm_noalloc(1, 8, 8, 8, 0, fake, fake, 0)
    assert e.value.code == ck.EINVAL


def _device_product(A, B, variant, stream):
    G, M, K = A.shape
    N = B.shape[1]
    dA = torch.from_numpy(A).to("cuda:0")
    dB = torch.from_numpy(B).to("cuda:0")
    dC = torch.full((G, M, N), complex(7.0, -7.0), dtype=torch.complex128, device="cuda:0")
    torch.cuda.synchronize()
    ck.ccsd_k_zgemm_noalloc(G, M, N, K, dA.data_ptr(), dB.data_ptr(), dC.data_ptr(), variant, stream.cuda_stream)
    stream.synchronize()
    return dC.cpu().numpy()


@pytest.mark.gpu
@pytest.mark.parametrize("variant", [0, 2])
def test_noalloc_matches_allocating_entry_point_twice(variant):
    rng = np.random.default_rng(11 + variant)
    stream = torch.cuda.Stream(device="cuda:0")  # default priority
    # first call: several tiles with ragged edges, K a multiple of 8 (the fast split path);
    # second call: smaller, K not a multiple of 8 (the gathered path)
    for (G, M, N, K) in [(3, 130, 200, 72), (2, 37, 45, 29)]:
        print(f"noalloc variant={variant} G={G} M={M} N={N} K={K}", flush=True)
        A = rng.standard_normal((G, M, K)) + 1j * rng.standard_normal((G, M, K))
        B = rng.standard_normal((G, N, K)) + 1j * rng.standard_normal((G, N, K))
        ref = ck.ccsd_k_debug_zgemm(A, B, reference=variant)
        got = _device_product(A, B, variant, stream)
        assert np.array_equal(got, ref), (G, M, N, K, np.abs(got - ref).max())
        # and the product itself is right (FP64 to rounding; split within its error model)
        exact = np.einsum("gmk,gnk->gmn", A, B)
        if variant == 0:
            assert np.abs(got - exact).max() <= 1e-13 * np.abs(exact).max() * K ** 0.5
        else:
            bound = np.einsum("gmk,gnk->gmn", np.abs(A), np.abs(B))
            assert np.all(np.abs(got - exact) <= 4e-5 * bound)
