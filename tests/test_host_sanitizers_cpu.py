"""The library's host code (construction by residues, canonical streams,
graph reader and labeller, code generation) built with g++ under
AddressSanitizer and UndefinedBehaviorSanitizer (every report aborts) and
driven over seeded diagrams of orders 2-6 in every construction mode, an
order-2 example, the seeded diagrams' graph files and malformed graph files
(tests/cpu_math/host_sanitize.cpp)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from ami_inputs import order2_example, random_self_energy

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2311_17189_amd", "csrc")


@pytest.mark.timeout(600)
def test_host_code_under_address_and_ub_sanitizers(tmp_path):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "host_sanitize")
    srcs = [os.path.join(CSRC, f) for f in ("construct.cpp", "graph.cpp", "codegen.cpp", "abi.cpp")]
    subprocess.run([cxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"),
                    os.path.join(HERE, "cpu_math", "host_sanitize.cpp"), *srcs, "-o", exe],
                   check=True, capture_output=True, text=True)
    ds = [order2_example()] + [random_self_energy(o, (0, o, i)) for o in (2, 3, 4, 5) for i in range(3)]
    ds.append(random_self_energy(6, (0, 6, 0)))
    lines = [str(len(ds))]
    for d in ds:
        lines.append(f"{d.alpha.shape[0]} {d.eps.shape[1]} {d.alpha.shape[1]} {d.n_int}")
        lines.append(" ".join(str(int(v)) for v in np.asarray(d.alpha).ravel()))
        lines.append(" ".join(str(int(v)) for v in np.asarray(d.eps).ravel()))
    graphs = []
    for j, d in enumerate(ds[1:6]):
        p = tmp_path / f"g{j}.txt"
        p.write_text("# seeded graph\n" + "\n".join(" ".join(str(int(v)) for v in row) for row in d.graph) + "\n")
        graphs.append(str(p))
    for j, text in enumerate(["0 1 1\n", "0 1 1 0 7\n", "a b c d\n", "0 -1 1 0\n", "", "# only a comment\n",
                              "0 1 2 0\n", "99999999999 1 1 0\n"]):
        p = tmp_path / f"bad{j}.txt"
        p.write_text(text)
        graphs.append(str(p))
    graphs.append(str(tmp_path / "missing.txt"))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    res = subprocess.run([exe] + graphs, input="\n".join(lines) + "\n", capture_output=True, text=True, env=env,
                         timeout=500)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
    assert "0 failures" in res.stdout
