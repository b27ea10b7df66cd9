"""Host-side pieces of bench.py: the code hash that keys stored counter
measurements ignores comments and whitespace, and follows code changes."""
import bench


def test_code_tokens_drop_comments_and_whitespace():
    src = "int a; // note\n/* block\n comment */ int  b =\n 2;"
    assert bench.code_tokens(src) == "int a; int b = 2;"


def test_hash_follows_code_not_comments(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2506_00167_amd" / "csrc"
    csrc.mkdir(parents=True)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setitem(bench.KERNEL_SOURCES, "probe", ["k.hip"])
    (csrc / "k.hip").write_text("int f() { return 1; }\n")
    h0 = bench.kernel_source_hash("probe")
    (csrc / "k.hip").write_text("// a comment\nint f()  {\n  return 1; /* same */ }\n")
    assert bench.kernel_source_hash("probe") == h0
    (csrc / "k.hip").write_text("int f() { return 2; }\n")
    assert bench.kernel_source_hash("probe") != h0

