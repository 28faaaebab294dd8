"""The C ABI used from plain C: the header and an example program compile as
C11 (CPU), and the program links against libvjboost.so and trains on the GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "c_example", "train_example.c")
LIBDIR = os.path.join(ROOT, "paper_1306_1467_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _compile(out, link):
    cc = shutil.which("gcc") or "cc"
    cmd = [cc, "-std=c11", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROCM, "include"), SRC]
    if link:
        cmd += ["-o", out, "-L", LIBDIR, "-lvjboost", "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
                f"-Wl,-rpath,{LIBDIR}", f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}"]
    else:
        cmd += ["-c", "-o", out]
    return subprocess.run(cmd, capture_output=True, text=True)


def test_header_and_example_compile_as_c11(tmp_path):
    r = _compile(str(tmp_path / "train_example.o"), link=False)
    assert r.returncode == 0, r.stderr


@pytest.mark.gpu
def test_example_trains_from_c(tmp_path):
    if not os.path.exists(os.path.join(LIBDIR, "libvjboost.so")):
        pytest.fail("libvjboost.so is not built")
    exe = str(tmp_path / "train_example")
    r = _compile(exe, link=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe, "900", "6"], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().splitlines()[-1].startswith("ok: 6 rounds over 900 windows")
