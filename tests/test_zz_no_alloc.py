"""The entry point that allocates nothing, against the context path (needs the GPU).

sts_step_static runs one gate step on the caller's device arrays with all
its working memory in the library's static device array. Its result must be
the one sts_load_terms + sts_apply_gate + sts_truncate give on a context
(same kernels: FP64 bit for bit, complex64 bit for bit too), on two calls in
a row, the second with a smaller input, so that what the first call left in
the static array cannot leak into the second. Sizes beyond the array's
limit are refused before anything runs.
"""
import sys

import numpy as np
import pytest

from paper_2607_07816_amd import circuits as C
from tests.helpers import random_state

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(120)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def context_step(keys, amps, n, qs, U, K, p, prec):
    from paper_2607_07816_amd import _lib
    with _lib.State(n, K=K, p=p, precision=prec, capacity=max(len(keys), K, 1024)) as st:
        st.load_terms(keys, amps)
        st.apply_gate(qs, U)
        st.truncate()
        k, a = st.read_terms()
        s = st.stats()
    return k, a, s


def static_step(keys, amps, n, qs, U, K, p, prec):
    import torch

    from paper_2607_07816_amd import _lib
    dev = torch.device("cuda")
    cdt = torch.complex128 if prec == "c128" else torch.complex64
    kin = torch.from_numpy(keys.astype(np.int64)).to(dev)
    ain = torch.from_numpy(amps.astype(np.complex128 if prec == "c128" else np.complex64)).to(dev)
    kout = torch.full((K,), -1, dtype=torch.int64, device=dev)
    aout = torch.zeros(K, dtype=cdt, device=dev)
    nout = torch.zeros(1, dtype=torch.int64, device=dev)
    stats = torch.zeros(2, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    _lib.step_static(n, K, p, prec, qs, U, kin.data_ptr(), ain.data_ptr(), len(keys), kout.data_ptr(),
                     aout.data_ptr(), nout.data_ptr(), stats.data_ptr(), stream.cuda_stream)
    torch.cuda.synchronize()
    cnt = int(nout.item())
    k = kout[:cnt].cpu().numpy().astype(np.uint64)
    a = aout[:cnt].cpu().numpy().astype(np.complex128)
    o = np.argsort(k, kind="stable")
    return k[o], a[o], stats.cpu().numpy()


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_static_step_equals_context_step(prec):
    rng = np.random.default_rng(77)
    # the second input is smaller and the second rule keeps fewer terms, so
    # what the first call left behind would show if it leaked
    for n, N, m, K, p in ((40, 60000, 2, 65536, 0.97), (30, 9001, 3, 5000, 0.0)):
        keys, amps = random_state(rng, n, N)
        if prec == "c64":
            amps = amps.astype(np.complex64).astype(np.complex128)
        qs = tuple(int(q) for q in rng.choice(n, size=m, replace=False))
        U = C.haar_unitary(rng, 1 << m)
        say(f"static step {prec} n={n} N={N} m={m} K={K} p={p}")
        kc, ac, sc = context_step(keys, amps, n, qs, U, K, p, prec)
        ks, as_, ss = static_step(keys, amps, n, qs, U, K, p, prec)
        assert np.array_equal(ks, kc)
        assert np.array_equal(as_.view(np.uint64), ac.view(np.uint64))
        assert ss[0] == sc["W"] and ss[1] == sc["kept_fraction"]
        say(f"  {len(ks)} terms, kept fraction {ss[1]:.12f}")


def test_static_step_refuses_beyond_its_limit():
    import torch

    from paper_2607_07816_amd import _lib
    d = torch.zeros(8, dtype=torch.int64, device="cuda")
    a = d.data_ptr()
    u = np.eye(2, dtype=np.complex128)
    lim = _lib.STATIC_MAX_TERMS
    with pytest.raises(_lib.CapacityError):
        _lib.step_static(20, lim + 1, 0.0, "c128", (0,), u, a, a, 4, a, a, a)
    with pytest.raises(_lib.CapacityError):
        _lib.step_static(20, 16, 0.0, "c128", (0,), u, a, a, lim + 1, a, a, a)
    with pytest.raises(_lib.StsError):
        _lib.step_static(20, 0, 0.5, "c128", (0,), u, a, a, 4, a, a, a)
