"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports every entry
point that include/deco.h declares, and its host utilities agree with the oracle."""
import os
import re

import numpy as np
import pytest

import oracle
from paper_2509_18612_amd import deco

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "deco.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(deco_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_named_entry_points():
    names = declared_functions()
    for required in ["deco_init", "deco_step", "deco_round_score", "deco_solve", "deco_best", "deco_start",
                     "deco_destroy", "deco_workspace_size", "deco_status_string"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    L = deco.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(deco.EXPORTS) == set(declared_functions())


def declared_param_counts():
    src = open(os.path.join(ROOT, "include", "deco.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    out = {}
    for name, params in re.findall(r"\b(deco_[a-z_0-9]+)\s*\(([^;{]*?)\)\s*;", src, flags=re.S):
        params = params.strip()
        out[name] = 0 if params in ("", "void") else params.count(",") + 1
    return out


def test_binding_argument_counts_match_the_header():
    """Every ctypes prototype of the binding takes as many arguments as the C declaration
    (a signature change on one side only would shift every later argument)."""
    L = deco.lib()
    counts = declared_param_counts()
    assert set(counts) == set(declared_functions())
    for name, k in counts.items():
        at = getattr(L, name).argtypes
        assert at is not None, f"{name} has no prototype"
        assert len(at) == k, (name, len(at), k)


def test_binding_structs_match_the_c_layout(tmp_path):
    """The ctypes structures of the binding have the C compiler's size and field offsets for
    every struct of the header (gcc compiles a probe against include/deco.h)."""
    import ctypes as ct
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("needs gcc")
    structs = [deco.deco_graph, deco.deco_params, deco.deco_start_args, deco.deco_schedule,
               deco.deco_solve_params, deco.deco_solve_report]
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "deco.h"', "int main(void) {"]
    for S in structs:
        lines.append(f'  printf("{S.__name__} size %zu\\n", sizeof({S.__name__}));')
        for f in S._fields_:
            lines.append(f'  printf("{S.__name__} {f[0]} %zu\\n", offsetof({S.__name__}, {f[0]}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = {}
    for ln in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        s_name, field, val = ln.split()
        got[(s_name, field)] = int(val)
    for S in structs:
        assert got[(S.__name__, "size")] == ct.sizeof(S), S.__name__
        for f in S._fields_:
            assert got[(S.__name__, f[0])] == getattr(S, f[0]).offset, (S.__name__, f[0])


def test_status_strings():
    for s in [0, -1, -2, -3, -4, -5, -6]:
        assert deco.status_string(s) and deco.status_string(s) != "unknown status"
    assert deco.status_string(-99) == "unknown status"


def test_host_philox_matches_published_vectors(golden_dir):
    with open(os.path.join(golden_dir, "philox4x32_10_kat.txt")) as f:
        for ln in f:
            if ln.startswith("#") or not ln.strip():
                continue
            t = [int(x, 16) for x in ln.split()]
            assert [int(x) for x in deco.philox(t[0:4], t[4:6])] == t[6:10]


@pytest.mark.parametrize("seed", [0, 1, 12345])
def test_evolution_step_matches_oracle_exactly(seed):
    rng = np.random.default_rng(seed)
    for rnd in range(5):
        K = 8
        fit = rng.integers(0, 5, K).astype(float)  # ties on purpose
        eq = rng.uniform(-4, -1, K)
        el = rng.uniform(-4, -1, K)
        lk = rng.integers(1, 5, K).astype(np.int32)
        a = deco.evo_next(fit, eq, el, lk, seed, rnd)
        b = oracle.evo_next(fit, eq, el, lk, seed, rnd)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("gene", [0, 1])
@pytest.mark.parametrize("seed", [0, 7, 98765])
def test_step_count_evolution_matches_oracle_exactly(seed, gene):
    rng = np.random.default_rng(seed)
    for rnd in range(5):
        K = 6
        fit = rng.integers(0, 4, K).astype(float)  # ties on purpose
        T = rng.integers(3000, 10001, K).astype(np.int32)
        a = deco.evo_next_steps(fit, T, 3000, 10000, seed, rnd, gene)
        b = oracle.evo_next_steps(fit, T, 3000, 10000, seed, rnd, gene)
        assert np.array_equal(a, b)
        order = sorted(range(K), key=lambda i: (-fit[i], i))
        assert np.array_equal(a[:K // 2], T[order[:K // 2]])
        for j in range(K // 2, K):
            t0 = T[order[j - K // 2]]
            assert max(3000, int(np.floor(t0 * 0.8))) <= a[j] <= min(10000, int(np.floor(t0 * 1.2)))


@pytest.mark.parametrize("seed", [0, 12345, 2**40 + 7])
def test_initial_population_matches_oracle_exactly(seed):
    """The solver's initial population (deco_evo_init) and the oracle's draw (Sec. 4.3) are
    bit-equal: exponents, lift dimensions and both step counts."""
    for K, lmax, tq, tl in [(8, 4, (3000, 10000), (100, 400)), (6, 1, (50, 50), (20, 20)), (64, 8, (1, 7), (9, 9))]:
        a = deco.evo_init(K, seed, lmax, tq, tl)
        b = oracle.evo_init(K, seed, lmax, tq, tl)
        for x, y in zip(a, b):
            assert x.dtype == y.dtype and np.array_equal(x, y)
    with pytest.raises(RuntimeError):
        deco.evo_init(4, 0, 4, (10, 9), (1, 1))


def test_step_count_genes_draw_apart():
    """The unlifted and lifted counts perturb with draws of their own: over a wide range the
    two genes' children differ, and a gene index past the lifted one is refused."""
    fit = np.arange(8, dtype=float)
    T = np.full(8, 50000, np.int32)
    a = deco.evo_next_steps(fit, T, 1, 100000, 3, 0, 0)
    b = deco.evo_next_steps(fit, T, 1, 100000, 3, 0, 1)
    assert np.array_equal(a[:4], b[:4]) and not np.array_equal(a[4:], b[4:])
    with pytest.raises(RuntimeError):
        deco.evo_next_steps(fit, T, 1, 100000, 3, 0, 2)


def test_workspace_size_and_argument_errors_without_device():
    g = deco.deco_graph(100, 400, 1, 1, None, 1, None)  # fake non-null pointers, never dereferenced
    import ctypes as ct
    nb = ct.c_size_t(0)
    p = deco.deco_params(16, 1, 0, 0, 0, 1, 0.1, 0)
    assert deco.lib().deco_workspace_size(ct.byref(g), ct.byref(p), ct.byref(nb)) == 0 and nb.value > 0
    bad = [deco.deco_params(3, 1, 0, 0, 0, 1, 0.1, 0),   # B = 3 unsupported
           deco.deco_params(16, 1 << 20, 1, 0, 0, 1, 0.1, 0),  # l B = 2^24 columns unsupported
           deco.deco_params(16, 2, 0, 0, 0, 1, 0.1, 0),  # l > 1 needs lifted rounding
           deco.deco_params(16, 1, 0, 7, 0, 1, 0.1, 0),  # bad gradient form
           deco.deco_params(16, 1, 0, 0, 0, 0, 0.1, 0),  # score_every = 0
           deco.deco_params(16, 1, 0, 0, 0, 1, float("nan"), 0)]
    want = [deco.E_UNSUPPORTED, deco.E_UNSUPPORTED, deco.E_INVAL, deco.E_INVAL, deco.E_INVAL, deco.E_NONFINITE]
    for q, w in zip(bad, want):
        assert deco.lib().deco_workspace_size(ct.byref(g), ct.byref(q), ct.byref(nb)) == w
    # more than 8 components: the workspace holds the column handle, the sum handle and two
    # n x B sum buffers
    w8, w9 = ct.c_size_t(0), ct.c_size_t(0)
    assert deco.lib().deco_workspace_size(ct.byref(g), ct.byref(deco.deco_params(16, 8, 1, 0, 0, 1, 0.1, 0)),
                                          ct.byref(w8)) == 0
    assert deco.lib().deco_workspace_size(ct.byref(g), ct.byref(deco.deco_params(16, 9, 1, 0, 0, 1, 0.1, 0)),
                                          ct.byref(w9)) == 0
    assert w9.value > w8.value > 0
    big = deco.deco_graph(100, 2 ** 31, 1, 1, None, 1, None)
    assert deco.lib().deco_workspace_size(ct.byref(big), ct.byref(p), ct.byref(nb)) == deco.E_UNSUPPORTED
    empty = deco.deco_graph(0, 0, 1, 1, None, 1, None)
    assert deco.lib().deco_workspace_size(ct.byref(empty), ct.byref(p), ct.byref(nb)) == deco.E_INVAL


def test_bits_round_trip():
    rng = np.random.default_rng(0)
    for B in [1, 2, 4, 8, 24, 64]:
        z = rng.integers(0, 2, (37, B)).astype(np.uint8)
        assert np.array_equal(deco.bits_to_z(deco.z_to_bits(z), B), z)
