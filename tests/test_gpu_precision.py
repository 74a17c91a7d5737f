"""Precision study on the K=16384, T=36, dt=5 ms contact workload at
lambda in {0.01, 0.1, 1}: FP64 and FP32 GPU rollouts against the FP64 CPU
oracle, same Philox counters.

For each lambda and each GPU mode the test prints the max / p99 / median
per-sample relative cost error, max |dS|/lambda (the weight-perturbation
scale), and max |dU_new| (N m) in both parity modes of the update (Eq. 4):
stage-isolated (oracle weighting of the GPU's own costs and noise) and
end-to-end (the oracle's own update).  FP32 rollouts are run with the Eq. 4
sums in FP64 (lambda below the switch-over threshold) and, as a contrast,
with the sums forced to FP32.

Bars: FP64 rollouts reach 1e-9 on every cost and 1e-3 N m end-to-end;
FP32 rollouts meet the FP32 cost criterion (1e-4, or kappa u32 for
ill-conditioned force estimates) and 1e-3 N m stage-isolated at every
lambda; end-to-end only where max |dS|/lambda <= 1e-3 (otherwise a
selection flip among near-tied samples is a precision finding that the
test reports with the top-2 cost gap).
"""
import numpy as np
import pytest

from paper_2609_02020_amd import binding as B
from gpu_util import U_ATOL, check_costs_fp32, cost_rel_err, device_update

pytestmark = pytest.mark.gpu
TICK = 4
K_FLAG_MAX = 80   # of 16384 samples, each within kappa u32 (checked one by one)

# (label, rollout precision, lambda threshold below which the Eq. 4 sums run in FP64)
MODES = [("fp64", B.FP64, 0.05), ("fp32+acc64", B.FP32, 0.05), ("fp32+acc32", B.FP32, 0.0)]


def test_precision_study(ora, workloads):
    rows = []
    for i, case in enumerate(workloads["precision_k16384"]):
        lam = case["cost"]["lambda"]
        print("precision_k16384[%d] lambda %g: oracle" % (i, lam), flush=True)
        st, U_ref, S_ref, _ = ora.update(case["robot"], case["cost"], case["target"], case["q0"],
                                         case["qd0"], case["U_nom"], case["seed"], TICK, want_noise=False)
        assert st == 0
        order = np.argsort(S_ref)
        gap = S_ref[order[1]] - S_ref[order[0]]
        for label, prec, thr in MODES:
            if label == "fp32+acc32" and lam >= 0.05:
                continue     # identical to fp32+acc64 above the threshold
            print("  mode %s" % label, flush=True)
            solver = B.Solver(case["robot"], case["cost"], prec, lambda_fp64_threshold=thr)
            out = device_update(solver, case, case["seed"], TICK, prec)
            solver.close()
            assert out["status"] == B.OK
            err = cost_rel_err(out["costs"], S_ref)
            st2, U_stage, _ = ora.weights_update(out["costs"], out["noise"], case["U_nom"], lam)
            assert st2 == 0
            dU_stage = np.abs(out["U_new"] - U_stage).max()
            dU_e2e = np.abs(out["U_new"] - U_ref).max()
            dS = np.abs(out["costs"] - S_ref).max() / lam
            flagged = []
            if prec == B.FP64:
                assert err.max() <= 1e-9, (label, lam, err.max())
                assert dU_e2e <= U_ATOL, (label, lam, dU_e2e)
            else:
                flagged = check_costs_fp32(ora, case, out["costs"], S_ref, case["seed"], TICK,
                                           "%s lambda %g" % (label, lam))
                assert len(flagged) <= K_FLAG_MAX
                if dS <= 1e-3:
                    assert dU_e2e <= U_ATOL, (label, lam, dU_e2e)
            assert dU_stage <= U_ATOL, (label, lam, dU_stage)
            rows.append((lam, label, err.max(), np.percentile(err, 99), np.median(err), dS,
                         dU_stage, dU_e2e, gap, len(flagged)))
    print("\n| lambda | mode | cost rel err max | p99 | median | max|dS|/lambda | "
          "|dU| stage (N m) | |dU| end-to-end (N m) | top-2 gap | kappa-flagged |")
    print("|---|---|---|---|---|---|---|---|---|---|")
    for r in rows:
        print("| %g | %s | %.3g | %.3g | %.3g | %.3g | %.3g | %.3g | %.3g | %d |" % r)
