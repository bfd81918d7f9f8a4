"""The C ABI without a GPU: symbols, struct layouts, error paths (CPU only)."""

import ctypes as C
import os
import re
import subprocess

import pytest

import paper_1612_09447_amd as pkg
from paper_1612_09447_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "eqs.h")


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(eqs_[a-zA-Z_0-9]+)\s*\(", src)))


def test_library_is_built():
    assert os.path.exists(binding.LIB_PATH), "run __graft_entry__.build() first"


def test_every_declared_symbol_is_exported():
    names = header_functions()
    assert len(names) >= 14
    out = subprocess.run(["nm", "-D", "--defined-only", binding.LIB_PATH], capture_output=True, text=True, check=True)
    exported = set(re.findall(r"\bT (eqs_\w+)", out.stdout))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    # and the binding declares a signature for each of them
    assert set(names) == set(binding._SIGNATURES)
    L = pkg.lib()
    for n in names:
        assert getattr(L, n) is not None


STRUCTS = {
    "eqs_material": ["eps_r", "kappa0", "e_s", "alpha", "nonlinear", "reserved"],
    "eqs_drive": ["amp", "freq", "phase"],
    "eqs_amg_params": ["precision", "coarse_max", "max_levels", "flexible", "theta", "jacobi_weight",
                       "smooth_weight"],
    "eqs_solve_stats": ["iters", "status", "relres"],
    "eqs_step_stats": ["stages", "total_iters", "max_iters", "min_iters", "not_converged", "guess_used",
                       "guess_fallbacks", "reserved", "max_relres", "train_loss"],
    "eqs_guess_params": ["kind", "window", "capacity", "warmup", "batch", "bf16", "guard", "add_threshold", "lr", "seed",
                         "init"],
    "eqs_adapt_params": ["atol", "rtol", "tau0", "tau_min", "tau_max", "s_max", "max_attempts"],
    "eqs_adapt_record": ["t", "tau", "err", "s", "accepted"],
    "eqs_adapt_stats": ["accepted", "rejected", "max_s", "not_converged", "stages", "cg_iters", "last_tau"],
    "eqs_info": ["n_nodes", "n_tets", "n_free", "nnz_M", "n_levels", "precision", "level_rows", "level_nnz",
                 "level_p_nnz", "level_r_nnz", "device_bytes", "workspace_bytes", "workspace_used"],
}


def test_struct_layouts_match_header(tmp_path):
    prog = ['#include <stdio.h>', '#include <stddef.h>', '#include "eqs.h"', "int main(void){"]
    for s, fields in STRUCTS.items():
        prog.append(f'printf("{s} %zu\\n", sizeof({s}));')
        for f in fields:
            prog.append(f'printf("{s}.{f} %zu\\n", offsetof({s}, {f}));')
    prog.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(prog))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True).stdout.splitlines())
    for s, fields in STRUCTS.items():
        cls = getattr(binding, s)
        assert int(out[s]) == C.sizeof(cls), s
        for f in fields:
            assert int(out[f"{s}.{f}"]) == getattr(cls, f).offset, (s, f)


def test_constants_match_header():
    src = open(HEADER).read()
    for name in ["EQS_OK", "EQS_ERR_INVALID_ARG", "EQS_ERR_STATE", "EQS_ERR_HIP", "EQS_ERR_NOT_CONVERGED",
                 "EQS_ERR_BREAKDOWN", "EQS_ERR_NONFINITE", "EQS_ERR_ALLOC", "EQS_MAX_DRIVES", "EQS_MLP_NPARAM",
                 "EQS_MAX_GRAPH_ITERS"]:
        m = re.search(r"#define\s+%s\s+\(?(-?\d+)\)?" % name, src)
        assert m and int(m.group(1)) == getattr(binding, name), name


def test_enums_match_header():
    """Precision, start-vector and kernel-class enums of the header against the
    binding's constants and name maps."""
    src = open(HEADER).read()
    vals = {m.group(1): int(m.group(2)) for m in re.finditer(r"(EQS_[A-Z0-9_]+)\s*=\s*(-?\d+)", src)}
    for name in ["EQS_PREC_FP64", "EQS_PREC_FP32", "EQS_GUESS_PREVIOUS", "EQS_GUESS_ZERO", "EQS_GUESS_GALERKIN",
                 "EQS_GUESS_MLP", "EQS_GUESS_MOR"]:
        assert vals[name] == getattr(binding, name), name
    kclass = {k: v for k, v in vals.items() if k.startswith("EQS_KCLASS_") and k != "EQS_KCLASS_COUNT"}
    assert sorted(kclass.values()) == list(range(vals["EQS_KCLASS_COUNT"]))
    assert sorted(binding.KCLASS.values()) == sorted(kclass.values())
    for name, v in binding.KCLASS.items():
        assert kclass["EQS_KCLASS_" + name.upper()] == v, name
    for name, v in binding.GUESS_KINDS.items():
        assert vals["EQS_GUESS_" + name.upper()] == v, name


def _no_gpu():
    try:
        import torch

        return not torch.cuda.is_available()
    except Exception:
        return True


@pytest.mark.skipif(not _no_gpu(), reason="checks the no-device error path")
def test_error_paths_without_device():
    L = pkg.lib()
    h = C.c_void_p()
    assert L.eqs_create(C.byref(h), 0, None) == binding.EQS_ERR_HIP
    assert L.eqs_last_error()  # a message is recorded
    assert L.eqs_create(None, 0, None) == binding.EQS_ERR_INVALID_ARG
    assert b"NULL" in L.eqs_last_error()
    assert L.eqs_destroy(None) == binding.EQS_OK
    assert L.eqs_last_error() == b""
    # a NULL context is refused before any device work
    assert L.eqs_apply_M(None, None, None) == binding.EQS_ERR_INVALID_ARG
    assert L.eqs_galerkin_start(None, 1, None, None, None, None, None) == binding.EQS_ERR_INVALID_ARG
    assert b"NULL" in L.eqs_last_error()
    assert L.eqs_galerkin_start_noalloc(None, 1, None, None, None, None, None) == binding.EQS_ERR_INVALID_ARG
    # the workspace calls
    nf, ws = C.c_int64(), C.c_int64()
    assert L.eqs_query(None, C.byref(nf), C.byref(ws)) == binding.EQS_ERR_INVALID_ARG
    assert L.eqs_set_workspace(None, None, 0) == binding.EQS_ERR_INVALID_ARG
    assert b"NULL" in L.eqs_last_error()
    assert L.eqs_set_graph_iters(None, 4) == binding.EQS_ERR_INVALID_ARG
    assert L.eqs_batch_set_graph_iters(None, 4) == binding.EQS_ERR_INVALID_ARG
    assert L.eqs_set_deterministic(None, 1) == binding.EQS_ERR_INVALID_ARG
    assert L.eqs_state_size(None, C.byref(nf)) == binding.EQS_ERR_INVALID_ARG
    assert L.eqs_state_save(None, None, 0) == binding.EQS_ERR_INVALID_ARG
    assert L.eqs_state_load(None, None, 0) == binding.EQS_ERR_INVALID_ARG
    with pytest.raises(pkg.EqsError) as ei:
        pkg.Context(0)
    assert ei.value.code == binding.EQS_ERR_HIP


def test_binding_fails_loudly_without_library(monkeypatch):
    monkeypatch.setattr(binding, "_lib", None)
    monkeypatch.setattr(binding, "LIB_PATH", "/nonexistent/libeqs.so")
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        binding.lib()
