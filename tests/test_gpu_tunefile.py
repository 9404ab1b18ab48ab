"""Persisted sweep tuning (HELM_TUNE_FILE): a second process launches what the first one tuned.

The first process tunes the coarse one-level ORAS sweep of a small two-level
problem and records the decision; the second reads it, reports the same
launch (helm_sweep_config) and appends nothing, since it did not tune; both
applications agree with each other bitwise.  A file whose entries name
launches that cannot run on the problem (a group the library does not have,
an unknown variant) is not trusted: the process tunes again.
"""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import json, sys
import numpy as np
sys.path.insert(0, sys.argv[1])
import inputs
from paper_2103_14921_amd import helm
from oracle.operator import fit_weights
WO = fit_weights()
W = {k: getattr(WO, k) for k in ("w1", "w2", "w3", "wm1", "wm2", "wm3", "wm4")}
shape = (28, 26, 24)
c = inputs.velocity_thrust_belt(*shape, h=25.0)
S = helm.Solver(shape, 25.0, c, 10.0, (5, 5, 5, 0), weights=W, parts=(2, 2, 2), overlap=2, levels=2)
R = inputs.random_field((20, S.nc), seed=77)
Z = S.apply_oras(R, level=1)
np.save(sys.argv[2], Z)
print(json.dumps(S.sweep_config(1, 20)), flush=True)
S.close()
'''


def _run(tmp_path, tag):
    env = dict(os.environ, HELM_TUNE_FILE=str(tmp_path / "tune.txt"))
    print("[case] tune-file child", tag, flush=True)
    out = subprocess.run([sys.executable, "-c", CHILD, ROOT, str(tmp_path / f"z{tag}.npy")], env=env,
                         capture_output=True, text=True, timeout=240)
    assert out.returncode == 0, out.stderr[-2000:]
    return json.loads(out.stdout.strip().splitlines()[-1])


def test_second_process_launches_the_recorded_sweep(tmp_path):
    import numpy as np
    cfg1 = _run(tmp_path, 1)
    lines = (tmp_path / "tune.txt").read_text().splitlines()
    assert cfg1["group"] > 0 and any(l.startswith("sweep ") for l in lines)
    cfg2 = _run(tmp_path, 2)
    assert cfg2 == cfg1
    assert (tmp_path / "tune.txt").read_text().splitlines() == lines  # nothing re-tuned
    assert np.array_equal(np.load(tmp_path / "z1.npy"), np.load(tmp_path / "z2.npy"))


def test_inadmissible_entries_are_retuned(tmp_path):
    import numpy as np
    _run(tmp_path, 1)
    good = (tmp_path / "tune.txt").read_text().splitlines()
    bad = []
    for l in good:
        f = l.split()
        if f[0] == "sweep":
            f[8], f[11] = "64", "7"  # group 64, variant 7: neither exists
        bad.append(" ".join(f))
    (tmp_path / "tune.txt").write_text("\n".join(bad) + "\n")
    cfg = _run(tmp_path, 3)
    after = (tmp_path / "tune.txt").read_text().splitlines()
    assert len(after) > len(bad)  # tuned again and recorded
    assert cfg["group"] in (8, 16, 32)
    z1, z3 = np.load(tmp_path / "z1.npy"), np.load(tmp_path / "z3.npy")
    assert np.linalg.norm(z3 - z1) <= 1e-10 * np.linalg.norm(z1)
