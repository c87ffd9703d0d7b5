"""CPU checks of the C ABI library: it loads, exports every symbol the header
declares, its host-only coin matches the oracle's bit for bit, and argument
validation rejects bad calls before touching a device.  No compute call
needs a GPU here."""

import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle as O
import paper_2411_00688_amd as T
from paper_2411_00688_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(tvs_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_library_exports_every_header_symbol():
    L = _lib.lib()
    names = header_functions()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # and the binding declares every one of them
    assert set(names) <= set(_lib.PROTOTYPES), set(names) - set(_lib.PROTOTYPES)


def test_coin_bitwise_equals_oracle():
    rng = np.random.default_rng(0)
    for _ in range(200):
        seed = int(rng.integers(0, 2**63))
        stream = int(rng.integers(0, 2**20))
        p = float(rng.choice([0.01, 0.05, 0.1, 0.3, 0.5, 0.99, 1.0, rng.uniform(1e-6, 1)]))
        for k in list(range(0, 50)) + [10**6, 2**40]:
            assert T.tvs_coin(seed, stream, k, p) == O.coin(seed, stream, k, p)
    assert T.tvs_coin(1, 2, 0, 0.0) == -1 and T.tvs_coin(1, 2, 0, 1.5) == -1
    assert T.tvs_coin(1, 2, -1, 0.5) == -1


def test_subset_draw_bitwise_equals_oracle():
    rng = np.random.default_rng(1)
    for _ in range(100):
        seed = int(rng.integers(0, 2**63))
        stream = int(rng.integers(0, 2**20))
        n = int(rng.choice([1, 2, 3, 7, 10, 18, 180, 1024]))
        for k in list(range(0, 40)) + [10**6, 2**40]:
            assert T.tvs_subset(seed, stream, k, n) == O.subset(seed, stream, k, n)
    assert T.tvs_subset(1, 2, 0, 0) == -1 and T.tvs_subset(1, 2, -1, 4) == -1
    assert T.tvs_subset(1, 2, 0, 1025) == -1


def test_null_arguments_are_rejected_without_a_device():
    L = _lib.lib()
    out = C.c_void_p()
    assert L.tvs_op_identity(None, 4, 4, C.byref(out)) == 1
    assert b"null context" in L.tvs_last_error()
    assert L.tvs_tv_prox(None, 0, 4, 4, None, 0.1, 1, 0, None, None, None) == 1
    assert L.tvs_proxskip(None, 0, None, None, None, None, None, None) == 1
    assert L.tvs_spdhgskip(None, 0, None, None, None, 4, None, None, None, None) == 1
    assert L.tvs_fgp_set_variant(None, 0, 4, 4, 0) == 1
    # variant table is host data
    n = T.tvs_fgp_variant_count()
    assert n >= 4
    shapes = [T.tvs_fgp_variant(i) for i in range(n)]
    assert all(tw > 0 and th > 0 and ts >= 1 for tw, th, ts in shapes)
    with pytest.raises(T.TvsError):
        T.tvs_fgp_variant(n)


def test_solver_parameter_validation_messages():
    """Parameter checks run before any device work, so a bogus op pointer is
    never dereferenced when the parameters are already invalid."""
    L = _lib.lib()
    P = _lib.tvs_params(alpha=0.1, step=1.0, dual_step=1.0, p=0.0, outer_iters=1,
                        inner_iters=1)
    st = _lib.tvs_state()
    rc = L.tvs_proxskip(None, 0, None, C.byref(st), C.byref(P), None, None, None)
    assert rc == 1


def test_learned_prox_parameter_count_and_null_checks():
    assert T.tvs_cnn_param_count() == O.cnn_param_count() == 19682
    L = _lib.lib()
    out = C.c_void_p()
    assert L.tvs_cnn_create(None, 0, C.byref(out)) == 1
    assert L.tvs_cnn_forward(None, 1, 4, 4, None, None, 0, None, None) == 1
    assert L.tvs_cnn_prox(None, 4, 4, None, 0.1, 0, 1e-3, 10, None, None, None, None) == 1


STRUCTS = ("tvs_params", "tvs_state", "tvs_report", "tvs_slice", "tvs_dual_rof_params",
           "tvs_solve_ext", "tvs_batch_params")


def test_header_compiles_as_c_and_matches_the_binding_layout(tmp_path):
    """A C99 program built against include/tvskip.h and linked with the
    library: every struct's size and field offsets equal the ctypes
    declarations of the binding, and the coin called from C equals the
    oracle's."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "tvskip.h"', 'int main(void) {']
    for s in STRUCTS:
        lines.append(f'    printf("{s} size %zu\\n", sizeof({s}));')
        for f, _ in getattr(_lib, s)._fields_:
            lines.append(f'    printf("{s} {f} %zu\\n", offsetof({s}, {f}));')
    lines.append('    printf("coin %d\\n", tvs_coin(12345u, 7u, 99, 0.3));')
    lines.append('    return 0;\n}')
    src = tmp_path / "abi.c"
    src.write_text("\n".join(lines) + "\n")
    libdir = os.path.dirname(_lib.LIB_PATH)
    exe = tmp_path / "abi"
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                        str(src), "-o", str(exe), "-L", libdir, "-ltvskip",
                        f"-Wl,-rpath,{libdir}"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {}
    for ln in out:
        parts = ln.split()
        if len(parts) == 3:
            got[(parts[0], parts[1])] = int(parts[2])
        elif len(parts) == 2:
            got[(parts[0], None)] = int(parts[1])
    for s in STRUCTS:
        cls = getattr(_lib, s)
        assert got[(s, "size")] == C.sizeof(cls), s
        for f, _ in cls._fields_:
            assert got[(s, f)] == getattr(cls, f).offset, (s, f)
    assert got[("coin", None)] == O.coin(12345, 7, 99, 0.3)
