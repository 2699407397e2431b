"""Checkpoint / restore through the C ABI: a run interrupted by rewl_save,
restored into a fresh context with rewl_load and continued must be
bit-identical to the uninterrupted run (every random number is a function
of seed, walker and attempt count, so the saved state is the whole state)."""
import os
import sys

import numpy as np
import pytest

from helpers import bits, gpu_from, progress

pytestmark = pytest.mark.gpu


_say = progress


def _cfg(seed=11):
    return dict(lattice=("bcc", 4, [1.0, 0.5]), windows=(-600.0, -100.0, 60, 3, 0.75, 2),
                schedule=(4, 5, 1.0, 2.0 ** -8, 20000, 12800), seed=seed)


def _snapshot(g, n_inst, n_w):
    out = []
    for i in range(n_inst):
        for w in range(n_w):
            st = g.walker(i, w)
            out.append((bits(g.lng(i, w)).tolist(), g.hist(i, w).tolist(), g.visited(i, w).tolist(),
                        {k: (bits(v).item() if isinstance(v, float) else v) for k, v in st.items()}))
        out.append(bits(g.config(i, 0)).tolist())
        out.append(np.asarray(g.exchange_stats(i)).tolist())
    return out


@pytest.mark.parametrize("mode", ["fp64_det", "fp32_de"])
def test_save_load_continues_bit_identically(mode, tmp_path):
    cfgs = [_cfg(11), _cfg(11)]
    n_w = 6
    _say("checkpoint", mode)
    a = gpu_from(cfgs, mode)
    a.run(10)
    ref = _snapshot(a, 2, n_w)
    ref_step = a.step()

    b = gpu_from(cfgs, mode)
    b.run(4)
    path = str(tmp_path / "ck.bin")
    b.save(path)
    b.close()
    c = gpu_from(cfgs, mode, seed=999)    # different seed: everything must come from the file
    c.load(path)
    assert c.step() == 4
    c.run(6)
    assert c.step() == ref_step
    assert _snapshot(c, 2, n_w) == ref


def test_load_rejects_other_configuration(tmp_path):
    from paper_1411_4212_amd.rewl import RewlError
    a = gpu_from(_cfg(), "fp32_de")
    a.run(1)
    path = str(tmp_path / "ck.bin")
    a.save(path)
    other = dict(_cfg(), windows=(-600.0, -100.0, 61, 3, 0.75, 2))
    b = gpu_from(other, "fp32_de")
    with pytest.raises(RewlError) as e:
        b.load(path)
    assert e.value.code == -7
    m = gpu_from(_cfg(), "fp64")
    with pytest.raises(RewlError):
        m.load(path)
    # truncated file: rejected, and the context is left usable
    with open(path, "rb") as f:
        data = f.read()
    with open(path, "wb") as f:
        f.write(data[: len(data) // 2])
    same = gpu_from(_cfg(), "fp32_de")
    with pytest.raises(RewlError) as e:
        same.load(path)
    assert e.value.code == -7
    same.run(1)
    assert same.step() == 1
