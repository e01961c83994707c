"""Host-side checks of the roofline work model that bench.py reports
(algorithmic bytes and flops per interior cell of each kernel kind), against
the operation and array counts of the method written out here by hand for
the 9-species / 21-reaction workload: four coarse Gauss-Lobatto nodes, four
fine sub-steps per coarse interval."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402

NS, NR, N1, R = 9, 21, 4, 4
# primitive fields a pass needs: u, v, w, T, p, mu, lambda, lambda/cp, the mean
# molecular weight and Y_k (X_k = Y_k Wbar / W_k; h_k a polynomial in T)
NU, NP = 5 + NS, 9 + NS


def test_direction_pass_bytes():
    m = bench.work_model(NS, NR, N1, R)
    # read U, the primitives and four velocity gradients; dU/dt read and written
    assert m["dir_y"][1] == m["dir_z"][1] == 8 * (NU + NP + 4 + 2 * NU) == 512
    # in the multirate coarse evaluations the x pass stores dU/dt unread
    assert m["dir_x"][1] == 8 * (NU + NP + 4 + NU) == 400
    # single-rate evaluations: every pass reads and writes dU/dt
    assert bench.work_model(NS, NR, N1, 0)["dir_x"][1] == 512


def test_fine_sweep_bytes_and_flops():
    split = bench.work_model(NS, NR, N1, R, fused=False)
    fused = bench.work_model(NS, NR, N1, R, fused=True)
    # two-kernel form: the sub-step kernel reads and writes U, reads the r
    # increments of every component and writes r new f2 values; the
    # quadrature pass reads the interval's coarse f1 values (n1 + the new left
    # node) and fine f2 values (r + 1) and writes the r increments
    assert split["mr_fine"][1] == 8 * (2 * NU + R * NU + R * NS) == 960
    assert split["mr_src"][1] == 8 * (NU * (N1 + 1) + NS * (R + 1) + R * NU) == 1368
    # one kernel: the increments never reach memory
    assert fused["mr_fine"][1] == 8 * (2 * NU + NU * (N1 + 1) + NS * (R + 1) + R * NS) == 1432
    assert fused["mr_fine"][0] == split["mr_fine"][0] + split["mr_src"][0]
    # per sub-step: 32 flops per species and 75 per reaction for the chemistry,
    # 12 per species plus 63 for the Newton solve, 2 per component for the update
    assert split["mr_fine"][0] == R * (32 * NS + 75 * NR + 12 * NS + 63 + 2 * NU)
