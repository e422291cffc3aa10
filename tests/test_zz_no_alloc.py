"""The active-set update without a workspace (oit_update_active_set_noalloc): its
outputs equal those of oit_update_active_set bit for bit, call after call on the
library's static per-GPU scratch, which keeps the previous call's contents."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2605_13855_amd import oit

DEV = "cuda"


def log(msg):
    print(msg, flush=True)


def outputs(n, acap, dcap):
    return {"idx": torch.full((acap,), -7, dtype=torch.int32, device=DEV),
            "na": torch.full((1,), -7, dtype=torch.int32, device=DEV),
            "didx": torch.full((dcap,), -7, dtype=torch.int32, device=DEV),
            "dsg": torch.full((dcap,), 5, dtype=torch.int8, device=DEV),
            "nd": torch.full((1,), -7, dtype=torch.int32, device=DEV)}


def run_both(score, label, mode, k, thresh, acap, dcap):
    n = score.numel()
    lab_ws, lab_na = label.clone(), label.clone()
    a, b = outputs(n, acap, dcap), outputs(n, acap, dcap)
    nb = oit.select_workspace_bytes(n)
    ws = torch.zeros(nb + 256, dtype=torch.uint8, device=DEV)
    ws = ws[(-ws.data_ptr()) % 256:][:nb]
    oit.update_active_set(score, n, mode, k, thresh, lab_ws, a["idx"], a["na"], a["didx"], a["dsg"], a["nd"], ws)
    status = torch.full((1,), -1, dtype=torch.int32, device=DEV)
    oit.update_active_set_noalloc(score, n, mode, k, thresh, lab_na, b["idx"], b["na"], b["didx"], b["dsg"],
                                  b["nd"], status)
    torch.cuda.synchronize()
    st_ws = oit.read_status(ws)
    na, nd = int(a["na"].item()), int(a["nd"].item())
    log(f"  n {n}, mode {mode}, k {k}: {na} active, {nd} label changes, status {st_ws} / {int(status.item())}")
    assert int(status.item()) == st_ws
    assert torch.equal(lab_ws, lab_na)
    for key in a:
        assert torch.equal(a[key], b[key]), key
    return na, nd, st_ws


def test_noalloc_selection_equals_workspace_selection():
    rng = np.random.default_rng(42)
    # first call at the scratch's maximum size, then smaller calls on the same scratch
    n1 = oit.NOALLOC_SELECT_MAX_N
    s1 = (rng.integers(0, 4000, size=n1) / 7.0).astype(np.float32)     # ties
    lab1 = (rng.random(n1) < 0.05).astype(np.uint8)
    k1 = n1 // 20
    na, nd, st = run_both(torch.tensor(s1, device=DEV), torch.tensor(lab1, device=DEV), oit.SELECT_TOPK, k1, 0.0,
                          k1, n1)
    assert na == k1 and nd > 0 and st == 0
    n2 = 5000
    s2 = (rng.integers(0, 50, size=n2) / 7.0).astype(np.float32)
    lab2 = (rng.random(n2) < 0.3).astype(np.uint8)
    na, nd, st = run_both(torch.tensor(s2, device=DEV), torch.tensor(lab2, device=DEV), oit.SELECT_TOPK, 250, 0.0,
                          250, n2)
    assert na == 250 and st == 0
    # threshold mode, and a label-change list too small: the overflow bit, the first entries
    n3 = 3001
    s3 = rng.exponential(size=n3).astype(np.float32)
    lab3 = (rng.random(n3) < 0.5).astype(np.uint8)
    na, nd, st = run_both(torch.tensor(s3, device=DEV), torch.tensor(lab3, device=DEV), oit.SELECT_THRESHOLD, 0,
                          1.0, n3, 100)
    assert st & oit.STATUS_DELTA_OVERFLOW and nd == 100
    # the status of the next call starts clear
    na, nd, st = run_both(torch.tensor(s2, device=DEV), torch.tensor(lab2, device=DEV), oit.SELECT_TOPK, 250, 0.0,
                          250, n2)
    assert st == 0
