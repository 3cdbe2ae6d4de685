"""GPU parity for the 64-model batch (694,359 nodes, 16,392,645 Gauss points
in one block-diagonal plan): sampled node rows of four models (the smallest,
the largest and two seeded others), FP64 and mixed, bit for bit against the
oracle's values for each model assembled on its own (stored as SHA-256 by
tests/golden/make_fixtures.py on the CPU; the batch is block diagonal, so a
model's rows carry the same values with columns offset by the model's first
dof)."""
import hashlib
import json
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def test_batch_rows_equal_oracle():
    import torch
    import paper_1802_04256_amd as rp
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "batch64_rows.json")))
    prob = W.named("batch64")
    print(f"[gpu case] batch64: models={prob.n_models} gps={prob.n_gp}", flush=True)
    plan = rp.Plan.from_problem(prob)
    row_ptr, col_idx = plan.build_pattern()
    row_ptr = row_ptr.cpu().numpy()
    col_idx = col_idx.cpu().numpy()
    for precision in ("fp64", "mixed"):
        K = plan.assemble(cell_E=prob.cell_E, nu=prob.nu, precision=precision).cpu().numpy()
        plan.status()
        for mod in ref["models"]:
            off = int(prob.node_off[mod["model"]])
            assert int(prob.node_off[mod["model"] + 1]) - off == mod["n_nodes"]
            for row in mod["rows"]:
                I = off + row["node"]
                a, b = row_ptr[3 * I], row_ptr[3 * I + 3]
                assert [int(row_ptr[3 * I + k] - a) for k in range(4)] == row["row_ptr"], (mod["model"], row["node"])
                assert _sha(col_idx[a:b] - 3 * off) == row["col_sha256"]
                assert _sha(K[a:b]) == row[f"{precision}_sha256"], (precision, mod["model"], row["node"])
