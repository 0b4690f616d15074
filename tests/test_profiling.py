"""The source hash that ties a committed counter summary to the trace kernel's
code: comments and layout do not change it, code does."""
from paper_2605_05635_amd import profiling as P

SRC = '''// header
int f(int a) {   /* the
   block */ return a + 1;   // tail
}
const char* s = "// kept /* too */";
char q = '\\'';
'''


def test_comments_and_layout_ignored():
    edited = SRC.replace("// header", "// another header").replace("/* the", "/* other")
    edited = edited.replace("int f(int a) {", "int   f(int a)\n{")
    assert P.code_tokens(edited) == P.code_tokens(SRC)


def test_code_and_literals_kept():
    t = P.code_tokens(SRC)
    assert '"// kept /* too */"' in t and "'\\''" in t
    assert "header" not in t and "block" not in t and "tail" not in t
    assert P.code_tokens(SRC.replace("a + 1", "a + 2")) != t


def test_trace_hash_is_stable():
    h = P.trace_source_hash()
    assert len(h) == 16 and h == P.trace_source_hash()
