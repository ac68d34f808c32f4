"""CPU checks of the benchmark's contract that need no GPU: it refuses more
than one GPU with a message, and the HBM traffic it reports comes from a
counter summary taken on the current source of the product kernel."""
import hashlib
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_counter_summary_matches_the_product_kernel_source():
    """The default workload's counter summary names the sha256 of the kernel
    source its counters were taken on; bench.py reports the traffic only while
    they agree, so a change to the kernel must come with a new counter run."""
    sys.path.insert(0, ROOT)
    import bench
    name = "penny3d_p2_384k"
    text = open(os.path.join(ROOT, "profiles", f"spmv_fp64_{name}.md")).read()
    sha = re.search(r"^source_sha256 = ([0-9a-f]{64})$", text, re.M).group(1)
    alg = int(re.search(r"^algorithmic_bytes_per_launch = (\d+)$", text, re.M).group(1))
    src = os.path.join(ROOT, "paper_1911_10275_amd", "csrc", "hf_kernels_spmv.hip")
    assert hashlib.sha256(open(src, "rb").read()).hexdigest() == sha
    traffic = bench.spmv_traffic(name)
    # scaled FETCH_SIZE + WRITE_SIZE bytes per launch: at least the algorithmic
    # bytes of one product and within 10% of them
    assert traffic is not None and alg <= traffic <= 1.1 * alg
    assert bench.spmv_traffic("no_such_workload") is None
