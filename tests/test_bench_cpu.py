"""Host logic of bench.py: the kernel-code hash that ties committed counter
summaries to the code they were taken for (comments and whitespace do not
count, every token does)."""
import bench


def test_kernel_code_ignores_comments_and_whitespace():
    a = "int f(int x) { // one\n  return x + 1; /* two\n three */ }\n"
    b = "int f(int x)\n{\n    return x + 1; // edited comment\n}\n"
    assert bench.kernel_code(a) == bench.kernel_code(b) == "intf(intx){returnx+1;}"


def test_kernel_code_sees_token_changes_and_keeps_literals():
    a = 'const char *s = "a // not a comment"; int y = 2;'
    b = 'const char *s = "a // not a comment"; int y = 3;'
    assert "//notacomment" in bench.kernel_code(a)
    assert bench.kernel_code(a) != bench.kernel_code(b)
    assert bench.kernel_code("x = '/' / 2; /* c */") == "x='/'/2;"


def test_kernel_sha_is_stable_for_the_tree():
    assert bench.kernel_sha() == bench.kernel_sha()
    assert len(bench.kernel_sha()) == 16


def test_oracle_rows_sums_the_oracle_rows():
    # the CPU baseline's task runner: the sum over (view, rows) tasks on several
    # workers equals the oracle's whole-image sums of those rows
    import numpy as np

    import oracle
    from paper_2007_00745_amd import workloads
    a = workloads.View(workloads.window_from_bounds(-2.0, 1.0, -1.2, 1.2, 24, 40), 24, 40, 200)
    b = workloads.View((-0.745, 0.113, 1e-3, 1e-3), 9, 31, 500)
    tasks = [(a, [r]) for r in range(0, 24, 3)] + [(b, [1, 4, 8])]
    want = int(oracle.render(a.window, a.m, a.n, a.max_iter, a.R)[0::3].sum(dtype=np.int64))
    want += int(oracle.render(b.window, b.m, b.n, b.max_iter, b.R)[[1, 4, 8]].sum(dtype=np.int64))
    for threads in (1, 3):
        total, secs = bench._oracle_rows(tasks, threads)
        assert total == want and secs >= 0.0
