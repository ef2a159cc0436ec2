"""The C ABI used from plain C: the example program compiles against
include/apsp.h with gcc and links libapsp.so (CPU); on a GPU it runs and
checks its own answer."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2310_03983_amd", "examples", "apsp_example.c")
PKG = os.path.join(ROOT, "paper_2310_03983_amd")


def build_example(tmp_path, native):
    exe = str(tmp_path / "apsp_example")
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"), SRC,
           "-L", PKG, "-lapsp", "-L", "/opt/rocm/lib", "-lamdhip64",
           f"-Wl,-rpath,{PKG}", "-Wl,-rpath,/opt/rocm/lib", "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


def test_example_compiles_as_c(native, tmp_path):
    exe = build_example(tmp_path, native)
    assert os.path.exists(exe)


@pytest.mark.gpu
def test_example_runs_on_gpu(native, dev, tmp_path):
    exe = build_example(tmp_path, native)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "example ok" in out.stdout and "path: 0 1 2 3 4 5" in out.stdout


@pytest.mark.gpu
def test_example_plans_with_the_shipped_model_file(native, dev, tmp_path):
    """The trained model, exported as text, loads through the C ABI alone and
    plans the same candidate as the Python-installed model."""
    import json
    from paper_2310_03983_amd import autotune
    exe = build_example(tmp_path, native)
    model_txt = os.path.join(PKG, "data", "costmodel_mlp.txt")
    out = subprocess.run([exe, model_txt], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    line = next(l for l in out.stdout.splitlines() if l.startswith("plan for n=16384"))
    autotune.install(json.load(open(os.path.join(PKG, "data", "costmodel_mlp.json"))))
    _, ch = native.apsp_plan(16384, 0.01)
    assert f"candidate {ch} " in line, line
