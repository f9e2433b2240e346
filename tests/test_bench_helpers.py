"""Host-side helpers of bench.py that turn rocprofv3 output into the profile summaries."""
import csv

import bench


def test_code_only_ignores_comments_and_spacing():
    a = "int f(int x) {  // the sum\n    return x + 1; /* one more */\n}\n"
    b = "int f(int x) {\n  return x + 1;\n}  // changed comment\n"
    c = "int f(int x) {\n  return x + 2;\n}\n"
    assert bench._code_only(a) == bench._code_only(b)
    assert bench._code_only(a) != bench._code_only(c)


def test_kernel_name_drops_void_and_arguments():
    n = "void svr::render_kernel<5, 0, 0, 8, false, true, 0>(svr::RenderArgs)"
    assert bench._kernel_name(n) == "svr::render_kernel<5, 0, 0, 8, false, true, 0>"
    assert bench._kernel_name("svr::upload_init(int*)") == "svr::upload_init"


def test_per_call_sums_the_kernels_of_one_call(tmp_path):
    """Counter values of the last `calls` dispatches of each kernel the call launches are
    summed per call; kernels of the family that were not launched are skipped."""
    path = tmp_path / "run_counter_collection.csv"
    rows = []
    for d in range(4):  # two calls of a split render: clear, march, finalise each
        rows.append(("void svr::split_clear_kernel(unsigned long long*, long)", 1.0 + d))
        rows.append(("void svr::render_split_kernel<0, 0, 8, false, true, 0>(svr::RenderArgs, int)",
                     100.0 + d))
        rows.append(("void svr::split_finalize_kernel<0>(svr::RenderArgs)", 10.0))
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Counter_Value"])
        w.writerows(rows)
    # last two dispatches of each: clear 3 + 4, march 102 + 103, finalise 10 + 10
    assert bench._per_call(str(path), "render_mip0", 2) == (7 + 205 + 20) / 2
