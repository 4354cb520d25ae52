"""Host logic of the counter summaries (no GPU): the source hash ignores
comments and layout, so that it marks counters stale only when the code
the compiler sees changes."""
from paper_1707_09898_amd import rocprof_summary as rs


def test_code_tokens_drop_comments_and_whitespace():
    a = "int a = 1; // note\n/* block\n comment */ float b =  2.0f;\n"
    b = "int a = 1;\nfloat b = 2.0f; // other note\n"
    assert rs.code_tokens(a) == rs.code_tokens(b) == "int a = 1; float b = 2.0f;"


def test_code_tokens_keep_string_and_char_literals():
    t = 'const char *s = "a // b /* c */"; char q = \'"\'; char e = \'\\\'\'; // tail'
    out = rs.code_tokens(t)
    assert '"a // b /* c */"' in out and "'\"'" in out and "tail" not in out


def test_code_tokens_see_code_changes():
    assert rs.code_tokens("x = a + b;") != rs.code_tokens("x = a - b;")


def test_source_hash_is_stable():
    assert rs.source_hash() == rs.source_hash()
    assert len(rs.source_hash()) == 16
