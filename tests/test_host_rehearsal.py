"""Host-only rehearsal of whole plans (CPU): recording, scheduling, the
upload's lowering of every descriptor and the launch sequence of an H-LU, with
the HIP runtime calls of the host code replaced by stubs that keep "device"
memory in host memory.  Built with UBSan (no recovery) and the libstdc++
assertions (single grids, and batches appended as the batch entry point
plans them); the driver checks that every copy, fill and launch's descriptors
lie inside one allocation, that every event waited for was recorded and none
is used after it is destroyed, and that every recorded item is launched
once."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1703_09085_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None or not os.path.isdir("/opt/rocm/include"):
        pytest.skip("needs g++ and the HIP headers")
    exe = str(tmp_path_factory.mktemp("rehearsal") / "driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=undefined", "-fno-sanitize-recover=all",
           "-D_GLIBCXX_ASSERTIONS", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-include", os.path.join(HERE, "host_rehearsal", "host_shim.h"),
           os.path.join(HERE, "host_rehearsal", "driver.cpp")] + \
          [os.path.join(CSRC, f) for f in ("planner.cpp", "program.cpp", "structure.cpp")] + \
          ["-lpthread", "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    return exe


@pytest.mark.parametrize("mode", [0, 1, 2])
@pytest.mark.parametrize("schedule,side,dims,leaf,kmax", [
    ("dataflow", 16, 3, 8, 96),
    ("waves", 40, 2, 8, 64),
    ("late", 12, 3, 8, 96),
])
def test_plan_host_path(driver, mode, schedule, side, dims, leaf, kmax):
    env = dict(os.environ, HM_SCHEDULE=schedule)
    r = subprocess.run([driver, str(side), str(dims), str(mode), str(leaf), str(kmax)], env=env,
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok"), r.stdout
    if schedule == "late":
        assert "late 1" in r.stdout


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_dataflow_over_budget_falls_back_to_waves(driver, mode):
    # 16^3 grid, leaf 8: the earliest-wave temporaries take 0.43-0.86 GB, the
    # dataflow schedule's 2.4-3.5 GB; with a 1 GB budget the dataflow attempt
    # is given up and the plan runs in waves, launching every item
    env = dict(os.environ, HM_SCHEDULE="dataflow", HM_TEMP_BUDGET_GB="1.0")
    r = subprocess.run([driver, "16", "3", str(mode), "8", "96"], env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "late 0, dataflow 0" in r.stdout, r.stdout
    assert r.stdout.strip().endswith("ok"), r.stdout


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_batch_plan_host_path(driver, mode):
    # six 3D grids (sides 12 down to 7, leaf 8) recorded on parallel threads
    # and appended, then scheduled in the dataflow schedule, whose estimated
    # starts and epochs are followed one appended part per thread
    env = dict(os.environ, HM_SCHEDULE="dataflow")
    r = subprocess.run([driver, "12", "3", str(mode), "8", "96", "6"], env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "dataflow 1" in r.stdout, r.stdout
    assert r.stdout.strip().endswith("ok"), r.stdout
