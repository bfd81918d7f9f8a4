"""Workload configurations as JSON files (``eqsgen/configs/<name>.json``).

A configuration names the recipe that builds a workload's inputs (mesh
resolution, seeds, for the batched workload the instance count, seeds and
sizes) and the settings it runs with: RKC stages s, steps, step size tau, the
CG tolerance, the precision of the AMG hierarchy and the start vector. Like
the rest of the package it holds input data only.
"""

from __future__ import annotations

import json
import os
from typing import List, Optional

from .cases import Case, case_batch, case_c0, case_c1, case_c2, case_p2

CONFIG_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "configs")

RECIPES = ("c0", "c1", "c2", "c3", "p2")
GUESSES = ("previous", "zero", "galerkin", "mor", "mlp")
REQUIRED = ("name", "recipe", "s", "steps", "tau", "rtol", "precision", "guess")
OPTIONAL = ("description", "n", "seed", "instances", "base_seed", "sizes", "mlp_init_seed")


def config_names() -> List[str]:
    return sorted(f[:-5] for f in os.listdir(CONFIG_DIR) if f.endswith(".json"))


def load_config(name_or_path: str) -> dict:
    """Read and check a configuration: a file path, or the name of one under
    ``eqsgen/configs``."""
    path = name_or_path if name_or_path.endswith(".json") else os.path.join(CONFIG_DIR, name_or_path + ".json")
    with open(path) as f:
        cfg = json.load(f)
    missing = [k for k in REQUIRED if k not in cfg]
    unknown = sorted(set(cfg) - set(REQUIRED) - set(OPTIONAL))
    if missing or unknown:
        raise ValueError(f"{path}: missing keys {missing}, unknown keys {unknown}")
    if cfg["recipe"] not in RECIPES:
        raise ValueError(f"{path}: recipe must be one of {RECIPES}")
    if cfg["recipe"] == "c3":
        for k in ("instances", "base_seed", "sizes"):
            if k not in cfg:
                raise ValueError(f"{path}: the batched recipe needs {k!r}")
    elif "n" not in cfg:
        raise ValueError(f"{path}: the recipe needs the mesh resolution 'n'")
    if cfg["precision"] not in ("fp64", "fp32"):
        raise ValueError(f"{path}: precision must be fp64 or fp32")
    if cfg["guess"] not in GUESSES:
        raise ValueError(f"{path}: guess must be one of {GUESSES}")
    if not (isinstance(cfg["s"], int) and 2 <= cfg["s"] <= 256):
        raise ValueError(f"{path}: s must be an integer in [2, 256]")
    if not (isinstance(cfg["steps"], int) and cfg["steps"] >= 1):
        raise ValueError(f"{path}: steps must be a positive integer")
    if not (cfg["tau"] > 0 and cfg["rtol"] > 0):
        raise ValueError(f"{path}: tau and rtol must be > 0")
    if cfg["guess"] == "mlp" and "mlp_init_seed" not in cfg:
        raise ValueError(f"{path}: the network start vector needs 'mlp_init_seed'")
    return cfg


def cases_from_config(cfg: dict, n: Optional[int] = None, instances: Optional[int] = None) -> List[Case]:
    """The workload's cases (one, or one per instance of the batched recipe)
    with the configuration's settings; n and instances shrink a workload for
    tests (same recipe and seeds, smaller mesh or fewer instances)."""
    r = cfg["recipe"]
    if r == "c3":
        cases = case_batch(instances or cfg["instances"], cfg["base_seed"], tuple(cfg["sizes"]))
    else:
        nn = n or cfg["n"]
        seed = cfg.get("seed", 1)
        cases = [{"c0": lambda: case_c0(nn), "c1": lambda: case_c1(nn, seed), "c2": lambda: case_c2(nn, seed),
                  "p2": lambda: case_p2(nn, seed)}[r]()]
    for c in cases:
        if r != "c3":
            c.name = cfg["name"]
        c.s, c.steps, c.tau, c.rtol, c.precision = cfg["s"], cfg["steps"], cfg["tau"], cfg["rtol"], cfg["precision"]
        c.meta["guess"] = cfg["guess"]
        if "mlp_init_seed" in cfg:
            c.meta["mlp_init_seed"] = cfg["mlp_init_seed"]
    return cases
