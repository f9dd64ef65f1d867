"""The C interface library loads and exports every function include/brng.h
declares; host-only entry points and argument checks work without a GPU."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
from paper_1412_4825_amd import binding as b

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "brng.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(brng_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_function_is_exported():
    names = _declared()
    assert "brng_create" in names and "brng_run_gibbs" in names
    lib = ctypes.CDLL(b.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(b.EXPORTS)


def test_struct_layouts_match_header(tmp_path):
    """ctypes layouts equal what a C compiler makes of include/brng.h."""
    classes = {"brng_config": b.brng_config, "brng_gibbs_desc": b.brng_gibbs_desc,
               "brng_lda_full_desc": b.brng_lda_full_desc,
               "brng_serve_config": b.brng_serve_config, "brng_serve_done": b.brng_serve_done,
               "brng_serve_stats": b.brng_serve_stats}
    fields = {k: [f[0] for f in c._fields_] for k, c in classes.items()}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "brng.h"', "int main(void){"]
    for st, fs in fields.items():
        lines.append('printf("%%zu\\n", sizeof(%s));' % st)
        for f in fs:
            lines.append('printf("%%zu\\n", offsetof(%s, %s));' % (st, f))
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    want = []
    for st, cls in classes.items():
        want.append(ctypes.sizeof(cls))
        want += [getattr(cls, f).offset for f in fields[st]]
    assert got == want


@pytest.mark.parametrize("window", [[100, 0, 0, 0], [256, 0, 0, 0], [513, 0, 0, 0]])
def test_bad_window_rejected_without_device(window):
    with pytest.raises(b.BrngError) as e:
        b.brng_create(1, 64, window)
    assert e.value.status == b.BRNG_E_ARG


def test_bad_config_rejected():
    for kw in (dict(n_chains=0), dict(layout=7), dict(prec=3)):
        args = dict(seed=1, n_chains=64, window=[512, 0, 0, 0])
        args.update(kw)
        with pytest.raises(b.BrngError):
            b.brng_create(**args)


def test_null_context_rejected():
    lib = b.lib()
    assert lib.brng_fill_base(None, 0) == b.BRNG_E_ARG
    assert lib.brng_run_gibbs(None, None, 0) == b.BRNG_E_ARG
    assert lib.brng_run_lda_full(None, None) == b.BRNG_E_ARG
    assert lib.brng_destroy(None) == b.BRNG_OK
    assert b.brng_status_string(b.BRNG_E_KIND_DISABLED).startswith("pool kind disabled")


def test_sort_by_length_matches_contract():
    rng = np.random.default_rng(0)
    steps = rng.integers(1, 30, size=5000).astype(np.int32)
    assert np.array_equal(b.brng_sort_by_length(steps), oracle.sort_by_length(steps))


def test_serve_arguments_checked_without_device():
    for kw in (dict(hbm_budget=0), dict(max_active=0), dict(tick_steps=0), dict(tick_sweeps=0)):
        args = dict(hbm_budget=1 << 20, max_active=4, tick_steps=8, tick_sweeps=1)
        args.update(kw)
        budget = args.pop("hbm_budget")
        with pytest.raises(b.BrngError) as e:
            b.brng_serve_open(budget, [0, 4096, 4096, 0], **args)
        assert e.value.status == b.BRNG_E_ARG
    with pytest.raises(b.BrngError) as e:
        b.brng_serve_open(1 << 20, [0, 100, 4096, 0])
    assert e.value.status == b.BRNG_E_ARG
    for fn, args in ((b._lib.brng_serve_progress, (None, 0)),
                     (b._lib.brng_serve_stats_get, (None, None))):
        assert fn(*args) == b.BRNG_E_ARG
    assert b._lib.brng_serve_close(None) == b.BRNG_OK
    t0 = b.brng_serve_now()
    assert b.brng_serve_now() >= t0 > 0


def test_static_run_refusals_without_device():
    """brng_run_gibbs_static refuses requests the fixed array cannot hold,
    resumed requests, bad launch shapes and disabled kinds before any HIP
    call (addresses below are never dereferenced)."""
    fake = 1 << 20
    big = b.gibbs_desc(b.BRNG_MODEL_NORMEXP, 64 * 4096, fake, max_steps=1, seed=1)
    with pytest.raises(b.BrngError) as e:
        b.brng_run_gibbs_static(big, [0, 4096, 4096, 0])
    assert e.value.status == b.BRNG_E_TOO_LARGE
    assert "static scratch" in str(e.value)
    # just above the limit: 8 MiB of N and E windows per 256 units of 4,096
    # entries, plus the unit records
    mb = b.STATIC_SCRATCH_MB
    units = (mb << 20) // (2 * 4096 * 4)
    edge = b.gibbs_desc(b.BRNG_MODEL_NORMEXP, 64 * units, fake, max_steps=1, seed=1)
    with pytest.raises(b.BrngError) as e:
        b.brng_run_gibbs_static(edge, [0, 4096, 4096, 0])
    assert e.value.status == b.BRNG_E_TOO_LARGE
    ok = b.gibbs_desc(b.BRNG_MODEL_NORMEXP, 64, fake, max_steps=1, seed=1)
    for desc, window, wpb, status in (
            (b.gibbs_desc(b.BRNG_MODEL_NORMEXP, 64, fake, max_steps=1, seed=1,
                          flags=b.BRNG_FLAG_RESUME), [0, 4096, 4096, 0], 4, b.BRNG_E_ARG),
            (b.gibbs_desc(b.BRNG_MODEL_NORMEXP, 64, fake, max_steps=1, seed=1, unit_base=1),
             [0, 4096, 4096, 0], 4, b.BRNG_E_ARG),
            (ok, [0, 4096, 4096, 0], 3, b.BRNG_E_ARG),
            (ok, [0, 4000, 4096, 0], 4, b.BRNG_E_ARG),
            (ok, [0, 0, 4096, 0], 4, b.BRNG_E_KIND_DISABLED)):
        with pytest.raises(b.BrngError) as e:
            b.brng_run_gibbs_static(desc, window, wpb=wpb)
        assert e.value.status == status
    assert b._lib.brng_run_gibbs_static(None, None, 4, None) == b.BRNG_E_ARG


def test_lda_full_units_matches_the_oracle_numbering():
    """Items a full-LDA corpus needs: topic blocks of 1,024 words, then the
    documents (the oracle's numbering of the same corpus)."""
    import oracle
    for K, V, D in ((64, 4096, 100), (64, 4097, 100), (1, 1 << 20, 0), (13, 300, 40),
                    (64, 50000, 16384), (3, 8192, 12)):
        assert b.brng_lda_full_units(K, V, D) == oracle.lda_full_units(K, V, D), (K, V, D)
    assert b.brng_lda_full_units(64, 4097, 100) == 64 * 5 + 100
    assert b.brng_lda_full_units(5, 0, 3) == 0
