"""The seeded input generators: numpy and torch streams agree byte for byte,
erasure masks have the requested weight, and streams are reproducible."""
import numpy as np
import torch

from paper_1404_3458_amd import synth


def test_mix64_reference_values():
    # splitmix64 with seed 0: the first outputs of the published generator
    assert synth.u64(0, 3).tolist() == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_numpy_and_torch_streams_agree():
    k = synth.key(1, 2, synth.DATA)
    for n in (1, 7, 8, 1000, 4099):
        a = synth.random_bytes(k, n)
        b = synth.random_bytes_torch(k, n).numpy()
        assert (a == b).all()
    t = torch.empty(5000, dtype=torch.uint8)
    synth.fill_random_torch(k, t, chunk_bytes=1024)
    assert (t.numpy() == synth.random_bytes(k, 5000)).all()


def test_erasure_mask_weight_and_determinism():
    for n, e in ((16, 8), (256, 128), (65536, 32768), (10, 0), (10, 10)):
        m = synth.erasure_mask(synth.key(5, n), n, e)
        assert m.sum() == e and m.dtype == np.uint8
        assert (m == synth.erasure_mask(synth.key(5, n), n, e)).all()


def test_uniform_int_range():
    v = synth.uniform_int(synth.key(9), 10000, 3, 7)
    assert v.min() == 3 and v.max() == 7


def test_mixed_stripes_shapes():
    sh = synth.mixed_stripes(4, 2000)
    assert sh == synth.mixed_stripes(4, 2000)           # reproducible
    classes = {(n, k) for n, k, _, _ in sh}
    assert classes == set(synth.MIXED_CLASSES)
    for n, k, sb, e in sh:
        assert 1024 <= sb <= 65536 and sb % 2 == 0
        assert 0 <= e <= n - k
    # log-uniform: about half the shards below the geometric mean 8 KiB
    below = sum(1 for _, _, sb, _ in sh if sb < 8192)
    assert 850 < below < 1150
