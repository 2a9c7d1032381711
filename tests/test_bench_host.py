"""Host-side checks of bench.py's accounting (no GPU).

The compulsory bytes per launch follow the per-unit figures of the kernels (64 B per
tet and 36 B per tile particle in the forward element pass, ...), recomputed here by
hand for the 256-body batch; measured HBM traffic is reported only for the kernel
source it was taken with; more than one GPU is refused with a message.
"""
import hashlib
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

NE, NP, NTP = 1367346, 307196, 676018  # the 256-body batch: tets, particles, tile particles


def test_kernel_bytes_per_unit():
    # one pass over one tet / one particle / one tile particle (T = K = 1: one forward pass)
    assert bench.kernel_bytes("element_fwd", 1, 0, 0, 1, 1) == 64
    assert bench.kernel_bytes("element_fwd", 0, 0, 1, 1, 1) == 36
    assert bench.kernel_bytes("element_adj", 1, 0, 0, 1, 1) == 80
    assert bench.kernel_bytes("element_adj", 0, 0, 1, 1, 1) == 69
    assert bench.kernel_bytes("particle_adj", 0, 1, 0, 1, 1) == 89
    # particle forward: 57 per particle and pass, plus one checkpoint store (24) per segment
    assert bench.kernel_bytes("particle_fwd", 0, 1, 0, 1, 1) == 57 + 24


def test_batch_bytes_per_launch():
    T, K = 100, 10
    fwd_launches = T + (T - T // K)  # rollout + recompute of 9 of every 10 steps
    assert fwd_launches == 190
    per = bench.kernel_bytes("element_fwd", NE, NP, NTP, T, K) / fwd_launches
    assert per == 64 * NE + 36 * NTP == 111846792
    # the first adjoint step stages the adjoint state (41 B per tile particle), the others
    # the adjoint force the previous particle adjoint stored (24 B)
    per_adj = bench.kernel_bytes("element_adj", NE, NP, NTP, T, K)
    assert per_adj == T * (80 * NE + 52 * NTP) + 17 * NTP


def test_shared_launch_bytes():
    """A shared launch (one adjoint and one recompute pass of the overlapped backward)
    counts both passes' algorithmic bytes; its compulsory bytes are both passes' less, for
    the element launch, the second read of the element records; a pass's compulsory bytes
    do not depend on how many of its passes run on their own."""
    T, K = 100, 10
    for kind in ("element", "particle"):
        assert bench.algorithmic_bytes(kind + "_dual", NE, NP, K) == (bench.algorithmic_bytes(kind + "_fwd", NE, NP, K)
                                                                      + bench.algorithmic_bytes(kind + "_adj", NE, NP, K))
    fwd = bench.compulsory_per_launch("element_fwd", NE, NP, NTP, T, K, 109)
    assert fwd == 64 * NE + 36 * NTP
    adj = bench.compulsory_per_launch("element_adj", NE, NP, NTP, T, K, 10)
    assert adj == (T * (80 * NE + 52 * NTP) + 17 * NTP) / T
    # one workgroup runs both passes of a tile: the element records are read once
    assert bench.compulsory_per_launch("element_dual", NE, NP, NTP, T, K, 90) == fwd + adj - 64 * NE
    # side by side (models with fewer tiles): each pass reads the records
    assert bench.compulsory_per_launch("element_dual", NE, NP, NTP, T, K, 90, paired=False) == fwd + adj
    pf = bench.compulsory_per_launch("particle_fwd", NE, NP, NTP, T, K, 100)
    pa = bench.compulsory_per_launch("particle_adj", NE, NP, NTP, T, K, 19)
    assert bench.compulsory_per_launch("particle_dual", NE, NP, NTP, T, K, 81) == pf + pa


def test_algorithmic_bytes():
    """The scope table's accounting: per launch, and for a whole checkpointed gradient
    (190 forward passes: 100 in the rollout, 90 recomputed)."""
    T, K = 100, 10
    assert bench.algorithmic_bytes("element_fwd", NE, NP, K) == 64 * NE + 12 * NP
    assert bench.algorithmic_bytes("particle_fwd", NE, NP, K) == 52 * NP
    assert bench.algorithmic_bytes("element_adj", NE, NP, K) == 64 * NE + 16 * NE / K + 40 * NP
    assert bench.algorithmic_bytes("particle_adj", NE, NP, K) == 84 * NP
    bf, ba = bench.step_algorithmic_bytes(NE, NP, K)
    assert bf == 64 * NE + 52 * NP and ba == 64 * NE + 84 * NP + 16 * NE / K
    assert 74 < bf / NE < 77 and 80 < ba / NE < 86  # the batch's ~75 B and ~84 B per element-step
    total, passes = bench.gradient_bytes(NE, NP, T, K)
    assert passes == 190 and total == 190 * bf + 100 * ba
    # the rollout's last segment kept for the backward: its 9 recompute passes do not run
    total, passes = bench.gradient_bytes(NE, NP, T, K, kept=True)
    assert passes == 181 and total == 181 * bf + 100 * ba
    assert bench.gradient_bytes(NE, NP, 1000, 50, kept=True)[1] == 1000 + 980 - 49
    assert bench.gradient_bytes(NE, NP, 40, 7, kept=True)[1] == 40 + 34 - 4  # ragged last segment of 5
    assert bench.gradient_bytes(NE, NP, 9, 10, kept=True)[1] == 9  # one segment: nothing recomputed
    # cloth: triangle 36 B, hinge 20 B per pass, stiffness gradient once per segment
    bf, ba = bench.step_algorithmic_bytes(0, 4096, 20, nt=7938, nh=11781)
    assert bf == 36 * 7938 + 20 * 11781 + 52 * 4096 and ba == bf + 32 * 4096 + 8 * 7938 / 20


def test_measured_traffic_only_for_its_source():
    h = hashlib.sha1()
    for name in ("gsim_kernels.hip", "gsim_device.h"):
        with open(os.path.join(ROOT, "paper_2104_02646_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    current = h.hexdigest() == bench.MEASURED_TRAFFIC["source_sha1"]
    v = bench.measured_traffic("element_fwd", 256, 100, 10, 512)
    assert (v == bench.MEASURED_TRAFFIC["per_launch"]["element_fwd"]) if current else v is None
    assert bench.measured_traffic("element_fwd", 128, 100, 10, 512) is None
    assert bench.measured_traffic("element_fwd", 256, 50, 10, 512) is None
    assert bench.measured_traffic("element_fwd", 256, 100, 10, 256) is None  # other tiles: other traffic


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120, env=dict(os.environ, HIP_VISIBLE_DEVICES=""))
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
