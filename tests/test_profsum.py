"""Host logic of the profile summaries: the digest that ties the committed
traffic counters to the kernel's sources ignores comments and layout, and
changes with the code."""
import os
import shutil

from paper_1812_10048_amd import profsum


def _digest_of(tmp_path, edit):
    """source_digest over copies of the traffic sources, one of them edited."""
    root = tmp_path / "pkg"
    for f in profsum.TRAFFIC_SOURCES:
        dst = root / f
        dst.parent.mkdir(parents=True, exist_ok=True)
        shutil.copy(os.path.join(profsum.HERE, f), dst)
    if edit:
        p = root / profsum.TRAFFIC_SOURCES[0]
        p.write_text(edit(p.read_text()))
    return profsum.source_digest([str(root / f) for f in profsum.TRAFFIC_SOURCES])


def test_digest_ignores_comments_and_whitespace(tmp_path):
    base = _digest_of(tmp_path, None)
    assert base == _digest_of(tmp_path, lambda t: t + "\n// a new comment\n/* and a block\n comment */\n")
    assert base == _digest_of(tmp_path, lambda t: t.replace("\n", "\n\n", 3))


def test_digest_changes_with_the_code(tmp_path):
    base = _digest_of(tmp_path, None)
    assert base != _digest_of(tmp_path, lambda t: t + "\nstatic int extra_symbol = 1;\n")


def test_code_only_strips_both_comment_forms():
    assert profsum._code_only("a = 1; // x\n/* y\n z */ b  =\t2;") == "a = 1; b = 2;"
