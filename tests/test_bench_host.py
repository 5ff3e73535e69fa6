"""Host logic of bench.py that runs without a GPU: the parsing of the system
management tools' JSON in the sustained-power probe."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

AMD_SMI = {"gpu_data": [{"gpu": 0,
                         "power": {"socket_power": {"value": 1352, "unit": "W"}, "throttle_status": "N/A"},
                         "clock": {"gfx_0": {"clk": {"value": 1746, "unit": "MHz"},
                                             "max_clk": {"value": 2400, "unit": "MHz"}}}}]}
ROCM_SMI = {"card0": {"Max Graphics Package Power (W)": "1400.0"}}


class _Done:
    def __init__(self, out):
        self.stdout = out
        self.returncode = 0


def _fake_run(outputs):
    def run(cmd, **kw):
        return _Done(outputs[cmd[0]])
    return run


def test_smi_reading_parses_both_tools(monkeypatch):
    # amd-smi prints more after its JSON object; the reader takes the first object only
    outs = {"amd-smi": json.dumps(AMD_SMI, indent=2) + "\n{\"cpu_data\": []}\n",
            "rocm-smi": "WARNING: a line before the JSON\n" + json.dumps(ROCM_SMI)}
    monkeypatch.setattr(subprocess, "run", _fake_run(outs))
    r = bench.smi_reading()
    assert r == {"socket_power_w": 1352, "gfx_clk_mhz": 1746, "power_cap_w": 1400.0}


def test_smi_reading_without_tools(monkeypatch):
    def missing(cmd, **kw):
        raise FileNotFoundError(cmd[0])
    monkeypatch.setattr(subprocess, "run", missing)
    assert bench.smi_reading() == {"socket_power_w": None, "gfx_clk_mhz": None, "power_cap_w": None}


def test_smi_reading_with_unexpected_output(monkeypatch):
    outs = {"amd-smi": "no devices found\n", "rocm-smi": json.dumps({"card0": {}})}
    monkeypatch.setattr(subprocess, "run", _fake_run(outs))
    assert bench.smi_reading() == {"socket_power_w": None, "gfx_clk_mhz": None, "power_cap_w": None}


def test_fp64_traffic_profile_taken_on_current_kernel():
    """The headline's HBM traffic comes from the committed counter summary only
    while that summary was taken on the current FP64 kernel code; this fails
    when the kernel changes and the counters have not been taken again."""
    t = bench.read_traffic("qgemm_f64_8192", bench.source_sha(*bench.FP64_SOURCES))
    assert t is not None and 8.59e9 < t < 1e12
