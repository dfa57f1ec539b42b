"""Host-side logic of bench.py that needs no GPU."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import bench  # noqa: E402


def test_code_digest_ignores_comments_and_whitespace(tmp_path):
    a = tmp_path / "a.hip"
    b = tmp_path / "b.hip"
    c = tmp_path / "c.hip"
    a.write_text("// header\nint f(int x) {\n  return x + 1;  /* one */\n}\n")
    b.write_text("/* other\n   header */\nint f(int x) { return x + 1; }  // same code\n")
    c.write_text("int f(int x) { return x + 2; }\n")
    assert bench.code_digest(str(a)) == bench.code_digest(str(b))
    assert bench.code_digest(str(a)) != bench.code_digest(str(c))


def test_committed_counters_match_the_kernel_code():
    """The committed HBM counter summary was taken on the kernel code in the tree, so bench.py reports
    its traffic for the dominant kernel (in the launch shape the counters were taken with)."""
    rest = [[3, 8, 1], [4, 16, 1], [3, 8, 1]]
    t32 = bench.measured_traffic("rhs_xdht", [[2, 4, 5]] + rest, 8, (256, 256, 256))
    t16 = bench.measured_traffic("rhs_xdht", [[2, 4, 4]] + rest, 8, (256, 256, 256))
    assert t16 is not None and t32 is not None and t16 > t32 > 0   # thinner z-chunks re-read more halo
    assert bench.measured_traffic("rhs_xdht", [[2, 8, 4]] + rest, 8, (256, 256, 256)) is None


def test_kernel_names_match_the_committed_trace():
    """bench.py's map from step kernels to device instantiations names kernels that the committed
    kernel trace of the 256^3 workload (taken at the shapes in its command) actually ran."""
    path = os.path.join(os.path.dirname(bench.__file__), "profiles", "step_sphere256_fp64_kernel_trace.md")
    text = open(path).read()
    shapes = [[int(v) for v in grp.split(",")] for grp in text.split('--shapes "')[1].split('"')[0].split(";")]
    names = {line.split("|")[1].strip() for line in text.splitlines() if line.startswith("| k_")}
    for step_kernel in ("rhs_xdht", "ydht_fwd", "neumann_solve", "ydht_inv", "xdht_out", "ghost_dphi", "ghost_fills"):
        for k in bench.kernel_template(step_kernel, shapes, 8, (256, 256, 256)):
            assert k in names, (step_kernel, k)
