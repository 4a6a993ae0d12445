"""GPU tests of the asynchronous particle copy (the store phase of the
paper's experiment, Section 4): each copy holds exactly the particles of the
step it was queued after, although stepping continues while it runs and the
record buffers are reused two propagations later; also inside a batch."""
import numpy as np
import pytest

from tests import _cases as C

pytestmark = [pytest.mark.gpu, pytest.mark.skip(
    reason="pf_copy_particles_async is switched off: its first GPU run (the first case below) "
           "ended in a GPU memory fault whose cause has not been found on the CPU")]


@pytest.fixture(scope="module")
def pf():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1212_1639_amd import pf as mod
    mod.lib()
    return mod


def _pinned(shape, dtype):
    import torch
    return torch.empty(shape, dtype=torch.float64 if dtype == np.float64 else torch.float32,
                       pin_memory=True)


@pytest.mark.parametrize("model,scheme,fp32", [("ll_pl", "stratified", True),
                                                ("sv_pl", "systematic", False),
                                                ("ll_pf", "multinomial", True)])
def test_copies_hold_each_steps_particles(pf, model, scheme, fp32):
    import torch
    n, T = 50000, 12
    print(f"async store {model} n={n} fp32={fp32}", flush=True)
    y = C.data(model, T)
    cfg = C.pf_config(pf, model, n, 4, scheme, fp32, keep_ancestors=False)
    f = pf.Filter(cfg)
    ref = pf.Filter(C.pf_config(pf, model, n, 4, scheme, fp32, keep_ancestors=False))
    shape, dt = f.record_shape()
    cs = torch.cuda.Stream()
    hosts = [_pinned(shape, dt) for _ in range(T)]
    for t in range(T):
        f.step(y[t])
        f.copy_particles_async(hosts[t], cs)
    cs.synchronize()
    torch.cuda.synchronize()
    for t in range(T):
        ref.step(y[t])
        rec, _, _ = ref.particles()
        np.testing.assert_array_equal(hosts[t].numpy(), rec)
    f.close()
    ref.close()


def test_copy_then_batch_step(pf):
    import torch
    sizes = [3000, 20000]
    T = 6
    y = np.stack([C.data("ll_pl", T, seed=k) for k in range(2)], axis=1)
    fs = [pf.Filter(C.pf_config(pf, "ll_pl", n, 9 + k, "stratified", True, keep_ancestors=False))
          for k, n in enumerate(sizes)]
    refs = [pf.Filter(C.pf_config(pf, "ll_pl", n, 9 + k, "stratified", True, keep_ancestors=False))
            for k, n in enumerate(sizes)]
    b = pf.Batch(fs)
    cs = torch.cuda.Stream()
    copies = []
    for t in range(T):
        b.step(y[t:t + 1])
        row = []
        for f in fs:
            shape, dt = f.record_shape()
            h = _pinned(shape, dt)
            f.copy_particles_async(h, cs)
            row.append(h)
        copies.append(row)
    cs.synchronize()
    torch.cuda.synchronize()
    for t in range(T):
        for k, r in enumerate(refs):
            r.step(y[t, k])
            rec, _, _ = r.particles()
            np.testing.assert_array_equal(copies[t][k].numpy(), rec)
    b.close()
    for f in fs + refs:
        f.close()


def test_copy_errors(pf):
    import torch
    f = pf.Filter(C.pf_config(pf, "ll_pl", 1000, 1, "stratified", True))
    small = torch.empty(10, dtype=torch.float32, pin_memory=True)
    with pytest.raises(AssertionError):
        f.copy_particles_async(small, torch.cuda.Stream())
    import ctypes
    rc = pf.lib().pf_copy_particles_async(f._h, ctypes.c_void_p(small.data_ptr()), 40, None)
    assert rc == pf.EINVAL
    f.close()
