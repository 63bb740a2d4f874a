"""Co-residency of the cooperative solve grid, proven from the compiler's
resource report (no GPU).

Every wave of the solve's grid must be resident at once: a wave that never
starts holds work items that resident waves wait on.  The library caps the
grid at 8 single-wave workgroups per compute unit and refuses more; this
test shows, from the gfx950 code object's own resource usage, that 8 fit:
no scratch memory, at most 256 VGPRs + AGPRs (2 waves on each of the CU's 4
SIMDs, 512 registers per lane each) and an occupancy of at least 2 waves per
SIMD in the compiler's own report, and 8 LDS rings within 160 KB even if LDS
were allocated in 2 KB granules."""
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2103_11445_amd", "csrc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
LDS_BYTES = 160 * 1024
GRANULE = 2048
WAVES_PER_CU = 8


def _resource_report():
    from paper_2103_11445_amd.build import HIP_FLAGS
    with tempfile.TemporaryDirectory() as tmp:
        r = subprocess.run([os.path.join(ROCM, "bin", "hipcc"), *HIP_FLAGS, "-c", os.path.join(CSRC, "solve.hip"),
                            "-o", os.path.join(tmp, "solve.o"), "-Rpass-analysis=kernel-resource-usage"],
                           capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    kernels, cur = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"remark:\s+Function Name: (\S+)", line)
        if m:
            cur = kernels.setdefault(m.group(1), {})
            continue
        m = re.search(r"remark:\s+([A-Za-z ]+?)(?: \[[^\]]*\])?: (\d+) \[", line)
        if m and cur is not None:
            cur[m.group(1).strip()] = int(m.group(2))
    return kernels


@pytest.fixture(scope="module")
def report():
    if not os.path.exists(os.path.join(ROCM, "bin", "hipcc")):
        pytest.skip("hipcc not available")
    return _resource_report()


def test_solve_kernels_prove_eight_waves_per_cu(report):
    solves = {k: v for k, v in report.items() if "solve_tiles" in k}
    assert len(solves) >= 8, sorted(report)
    for name, r in solves.items():
        assert r["ScratchSize"] == 0, name
        regs = r["VGPRs"] + r.get("AGPRs", 0)
        per_simd = 512 // (-(-regs // 8) * 8)
        assert 4 * per_simd >= WAVES_PER_CU, (name, regs)
        # and the compiler's own figure (it also counts what the register
        # count alone does not show)
        assert 4 * r["Occupancy"] >= WAVES_PER_CU, (name, r["Occupancy"])
        lds = -(-r["LDS Size"] // GRANULE) * GRANULE
        assert WAVES_PER_CU * lds <= LDS_BYTES, (name, r["LDS Size"])


def test_set_launch_refuses_unproven_shapes():
    import paper_2103_11445_amd as sp
    sp.load()
    import workloads as wl
    s = wl.stencil2d(10, seed=0)
    plan = sp.Plan(s.row_ptr, s.col_idx, s.val)
    for w in (0, 1, 8):
        plan.set_launch(w)
    with pytest.raises(sp.SptrsvError) as e:
        plan.set_launch(9)
    assert e.value.status == "ERR_ARG"
    plan.close()
