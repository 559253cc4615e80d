"""Host checks of the study fixtures: the oracle generator of tests/golden restates the
cells of the GPU studies (Sec. 3) with the same sizes, laws and seeds, and its stored
file holds every cell."""
import importlib.util
import json
import os

from paper_2311_03824_amd import studies as S

HERE = os.path.dirname(os.path.abspath(__file__))


def _generator():
    spec = importlib.util.spec_from_file_location("make_study_oracle", os.path.join(HERE, "golden", "make_study_oracle.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_generator_cells_are_the_studies_cells():
    g = _generator()
    assert g.FIG1 == S.FIG1 and g.FIG2 == S.FIG2 and g.TABLE1 == S.TABLE1 and g.SEED == S.SEED


def test_stored_oracle_errors_cover_every_cell():
    with open(os.path.join(HERE, "golden", "study_oracle.json")) as f:
        d = json.load(f)
    runs, runs_decided = d["runs_per_cell"], d["runs_rounding_decided"]
    assert 1 <= runs <= runs_decided
    assert sorted(d["fig1"]) == sorted(f"rho={r}" for r in S.FIG1["rhos"])
    assert sorted(d["fig2"]) == sorted(name for name, _, _ in S.FIG2["laws"])
    for n1, n2 in S.TABLE1["frames"]:
        assert sorted(d["table1"][f"{n1}x{n2}"]) == sorted(f"m={m}" for m in S.TABLE1["ms"])
    for cell in list(d["fig1"].values()) + list(d["fig2"].values()):
        assert len(cell) == runs and all(0.0 <= r["error"] < 1.0 for r in cell)
    for frame in d["table1"].values():
        for cell in frame.values():
            assert len(cell["runs"]) == (runs_decided if cell["rounding_decided"] else runs)
            assert all(0.0 <= r["error"] < 1.0 for r in cell["runs"])
            assert all("error_fp32_dft" in r for r in cell["runs"][:runs])
    # the oracle reproduces the paper's qualitative claims on these runs: exact recovery
    # (to the FP32 rounding of y) at rho = 2 in Fig. 1, and an error that falls with m in Table 1
    assert all(r["error"] < 1e-6 for r in d["fig1"]["rho=2"])
    for frame in d["table1"].values():
        means = [sum(r["error"] for r in frame[f"m={m}"]["runs"][:runs]) / runs for m in S.TABLE1["ms"]]
        assert means[0] > means[3] > means[4]
        # up to m = 100 the error after T_max iterations is set by how far U has
        # converged, and rounding leaves it alone
        assert not any(frame[f"m={m}"]["rounding_decided"] for m in S.TABLE1["ms"] if m <= 100)
