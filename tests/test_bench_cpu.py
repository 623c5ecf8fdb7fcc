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
