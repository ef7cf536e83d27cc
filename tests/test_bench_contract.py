"""bench.py on the CPU: more than one GPU is refused with a message, and the
committed rocprofv3 counters are used only while the kernels' sources (their
code, not their comments) are the ones they were taken from."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_source_hash_ignores_comments_and_whitespace():
    code = "int f(int a) {\n  return a + 1;  // one more\n}\n"
    same = "/* header */ int f(int a) { return a + 1; }\n"
    other = "int f(int a) { return a + 2; }"
    assert bench._code_only(code) == bench._code_only(same)
    assert bench._code_only(code) != bench._code_only(other)


def test_counters_follow_the_source_hash(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"traffic": {"fif::query_info_pipe_kernel": {"GB_per_launch": 22.4,
                                                        "src_hash": bench.query_src_hash()},
                       "fif::pc_kernel<1, false>": {"GB_per_launch": 0.5,
                                                    "src_hash": bench.src_hash(bench.PC_SOURCES)}},
           "flops": {"fif::build_kernel<1, 0>": {"fp32": 1e13, "src_hash":
                                                 bench.src_hash(bench.BUILD_SOURCES)}}}
    (prof / "counters.json").write_text(json.dumps(rec))
    real_join = os.path.join

    def join(*parts):  # point only the counters file at the temporary copy
        if len(parts) == 3 and parts[1] == "profiles" and parts[2] == "counters.json":
            return str(prof / "counters.json")
        return real_join(*parts)

    monkeypatch.setattr(bench.os.path, "join", join)
    assert bench.counter_traffic("fif::query_info_pipe_kernel") == 22.4e9
    assert bench.counter_traffic("fif::pc_kernel<1, false>") == 0.5e9
    assert bench.counter_flops("fif::build_kernel<1, 0>", bench.BUILD_SOURCES)["fp32"] == 1e13
    # each kernel's counters follow its own sources
    rec["traffic"]["fif::query_info_pipe_kernel"]["src_hash"] = "0" * 16
    rec["flops"]["fif::build_kernel<1, 0>"]["src_hash"] = "0" * 16
    (prof / "counters.json").write_text(json.dumps(rec))
    assert bench.counter_traffic("fif::query_info_pipe_kernel") is None
    assert bench.counter_traffic("fif::pc_kernel<1, false>") == 0.5e9
    assert bench.counter_flops("fif::build_kernel<1, 0>", bench.BUILD_SOURCES) is None
    assert bench.sources_of("fif::gp_query_trace_kernel<float>") == bench.GP_SOURCES
    assert bench.sources_of("fif::build_kernel<1, 1>") == bench.BUILD_SOURCES


def test_morton_key_of_the_sorted_leg():
    """The sorted-order leg's key interleaves the cell's x, y, z bits (x lowest);
    checked against a bit-by-bit interleave."""
    import numpy as np
    import torch

    rng = np.random.default_rng(5)
    cells = rng.integers(0, 1024, size=(500, 3))
    t = torch.from_numpy(cells).to(torch.int64)
    key = (bench._spread10(t[:, 0]) | (bench._spread10(t[:, 1]) << 1)
           | (bench._spread10(t[:, 2]) << 2)).tolist()
    for (i, j, k), got in zip(cells.tolist(), key):
        want = 0
        for b in range(10):
            want |= ((i >> b) & 1) << (3 * b) | ((j >> b) & 1) << (3 * b + 1) \
                | ((k >> b) & 1) << (3 * b + 2)
        assert got == want


def test_committed_bench_line_has_the_contract_keys():
    """The bench line kept under profiles/ carries every key of the JSON contract,
    including the roofline and CPU-baseline objects."""
    line = open(os.path.join(ROOT, "profiles", "bench_building_10M.json")).read()
    d = json.loads(line.strip().splitlines()[-1])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["value"] > 0 and "workload" in d["config"]
    r = d["roofline"]
    assert r["bound"] in ("hbm", "mfma", "alu") and r["unit"] in ("GB/s", "TFLOP/s")
    assert abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-9 and "traffic" in r
    c = d["cpu_baseline"]
    assert c["kind"] == "oracle" and c["cores"] >= 1 and c["value"] > 0 and c["sample"]
