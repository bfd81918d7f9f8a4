"""The JSON workload configurations (eqsgen/configs) against the recipes they
name: each holds the recipe's own settings (stages, steps, step size, CG
tolerance, precision; the network's seed for the learned form), builds the
same inputs (checked at reduced size: same recipe and seeds, smaller mesh or
fewer instances), and malformed files are refused. CPU only."""

import json

import numpy as np
import pytest

import eqsgen

ARRAYS = ("xyz", "tets", "tet_mat", "eps_r", "kappa0", "e_s", "alpha", "nonlinear", "dir_nodes", "dir_drive", "amp",
          "freq", "phase")


def recipe_case(cfg, n=None, instances=None):
    r = cfg["recipe"]
    if r == "c0":
        return [eqsgen.case_c0(n or cfg["n"])]
    if r == "c1":
        return [eqsgen.case_c1(n or cfg["n"], cfg["seed"])]
    if r == "c2":
        return [eqsgen.case_c2(n or cfg["n"], cfg["seed"])]
    if r == "p2":
        return [eqsgen.case_p2(n or cfg["n"], cfg["seed"])]
    return eqsgen.case_batch(instances or cfg["instances"], cfg["base_seed"], tuple(cfg["sizes"]))


def test_every_workload_has_a_configuration():
    assert eqsgen.config_names() == ["c0", "c1", "c2", "c3", "c4", "p2"]


@pytest.mark.parametrize("name", ["c0", "c1", "c2", "c3", "c4", "p2"])
def test_configuration_matches_its_recipe(name):
    cfg = eqsgen.load_config(name)
    small = dict(n=3) if cfg["recipe"] != "c3" else dict(instances=2)
    ref = recipe_case(cfg, **small)
    got = eqsgen.cases_from_config(cfg, **small)
    assert len(got) == len(ref)
    for a, b in zip(got, ref):
        # the recipe's own settings, unchanged by the file
        assert (a.s, a.steps, a.tau, a.rtol, a.precision) == (b.s, b.steps, b.tau, b.rtol, b.precision)
        for k in ARRAYS:
            np.testing.assert_array_equal(getattr(a, k), getattr(b, k), err_msg=k)
    if name == "c4":
        assert cfg["guess"] == "mlp" and cfg["mlp_init_seed"] == 4
    else:
        assert cfg["guess"] == "previous"
    if name in ("c2", "c4", "p2"):
        # the full-size mesh the file names: (m)^3 nodes less the two driven faces, 2,113,407 free DOF
        m = 2 * cfg["n"] + 1 if cfg["recipe"] == "p2" else cfg["n"] + 1
        assert m ** 3 - 2 * m * m == 2_113_407


@pytest.mark.parametrize("edit,msg", [
    (lambda c: c.pop("rtol"), "missing"),
    (lambda c: c.update(colour="red"), "unknown"),
    (lambda c: c.update(precision="fp16"), "precision"),
    (lambda c: c.update(s=1), "s must"),
    (lambda c: c.update(guess="mlp"), "mlp_init_seed"),
    (lambda c: c.update(recipe="c9"), "recipe"),
])
def test_malformed_configuration_is_refused(tmp_path, edit, msg):
    cfg = eqsgen.load_config("c2")
    edit(cfg)
    p = tmp_path / "bad.json"
    p.write_text(json.dumps(cfg))
    with pytest.raises(ValueError, match=msg):
        eqsgen.load_config(str(p))
