"""The GPU generator against the oracle's: Philox words bitwise on 10^6
counters, Box-Muller increments to FP32 accuracy."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_philox_words_bitwise(fk, oracle_mod):
    import torch
    rng = np.random.default_rng(42)
    n = 1 << 20
    ctr = rng.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:1024] = 0
    ctr[:1024, 0] = np.arange(1024)
    for seed in (0, 1, 0xDEADBEEFCAFEF00D):
        print(f"[gpu] philox n={n} seed={seed:#x}", flush=True)
        got = fk.fk_philox_words(torch.from_numpy(ctr.view(np.int32)).cuda(), seed).cpu().numpy().view(np.uint32)
        keys = np.tile(np.array([[seed & 0xFFFFFFFF, seed >> 32]], dtype=np.uint32), (n, 1))
        ref = oracle_mod.philox(ctr, keys)
        assert np.array_equal(got, ref)


def test_normals_match_oracle(fk, oracle_mod):
    import torch
    rng = np.random.default_rng(7)
    n = 1 << 20
    ra = rng.integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32)
    rb = rng.integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32)
    # the extremes of the 23-bit uniforms: m = 0 and m = 2^23 - 1 in each word
    ra[:4] = [0, 0x7FFFFF, 0xFF800000, 0xFFFFFFFF]
    rb[:4] = [0, 1 << 21, 0x7FFFFF, 0xFF800000]
    for D in (1e-5, 1e-4, 2.5e-5):
        print(f"[gpu] normals n={n} D={D}", flush=True)
        got = fk.fk_normals(torch.from_numpy(ra.view(np.int32)).cuda(), torch.from_numpy(rb.view(np.int32)).cuda(),
                            D).cpu().numpy().astype(np.float64)
        ref = oracle_mod.normals(ra, rb) * np.sqrt(2 * D)
        err = np.abs(got - ref) / np.sqrt(2 * D)
        print(f"max abs err / sqrt(2D) = {err.max():.3e}", flush=True)
        assert err.max() < 2e-6
