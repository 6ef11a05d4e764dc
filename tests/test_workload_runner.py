"""Named workloads: their initial fields and the command-line runner (paper_1505_06900_amd.run).

CPU: initial_fields gives each small workload the fields of its own recipe; the
runner refuses unknown names and bad step counts.  GPU: the runner's JSON records
of a short 64^3 Taylor-Green run (mass conserved to rounding, energy decaying,
step counts and rates present)."""
import json

import numpy as np
import pytest

import workloads as W


@pytest.mark.parametrize("name", ["tgv2d_64", "tgv3d_64_ma01", "tgv3d_64_ma05"])
def test_initial_fields_follow_the_recipe(name):
    cfg = W.WORKLOADS[name]
    rho, u, shape = W.initial_fields(name)
    ref = W.tgv2d(cfg["n"], cfg["u0"]) if cfg["lattice"] == "D2Q9" else W.tgv3d(cfg["n"], cfg["u0"])
    assert shape == ((1, 64, 64) if cfg["lattice"] == "D2Q9" else (64, 64, 64))
    assert rho.shape == shape and u.shape == (len(shape) if cfg["lattice"] != "D2Q9" else 2,) + shape
    np.testing.assert_array_equal(rho, np.asarray(ref[0]).reshape(shape))
    np.testing.assert_array_equal(u, np.asarray(ref[1]).reshape(u.shape))


def test_initial_fields_refuse_a_workload_without_a_recipe():
    with pytest.raises(KeyError):
        W.initial_fields("turb2d_coarse_256")


@pytest.mark.parametrize("argv", [["no_such_workload"], ["tgv2d_64", "--steps", "-1"],
                                  ["tgv2d_64", "--report-every", "0"], ["tgv2d_64", "--storage", "bf16"]])
def test_runner_rejects_bad_arguments(argv):
    from paper_1505_06900_amd import run

    with pytest.raises(SystemExit) as e:
        run.main(argv)
    assert e.value.code == 2


@pytest.mark.gpu
def test_runner_records(lbrr, gpu, capsys):
    from paper_1505_06900_amd import run

    assert run.main(["tgv3d_64_ma01", "--steps", "40", "--report-every", "20", "--storage", "fp32"]) == 0
    recs = [json.loads(line) for line in capsys.readouterr().out.splitlines() if line.startswith("{")]
    assert [r["step"] for r in recs] == [0, 20, 40]
    assert recs[0]["glups"] is None and all(r["glups"] > 0 for r in recs[1:])
    m0 = recs[0]["mass"]
    assert m0 == pytest.approx(64 ** 3, rel=1e-12)
    assert all(abs(r["mass"] - m0) <= 1e-9 * m0 for r in recs)
    ke = [r["kinetic_energy"] for r in recs]
    assert ke[0] > ke[1] > ke[2] > 0.9 * ke[0]
    assert all(abs(p) <= 1e-9 * m0 for r in recs for p in r["momentum"])
