"""Host logic of bench.py that needs no GPU.

The measured HBM traffic in the committed counter summary is reported only while
the kernel sources hash to the ones the counters were taken with; the hash is over
the code with comments and blank space removed, so editing a comment keeps it and
changing code (a string literal included) does not.
"""
import bench


def test_code_tokens_drop_comments_only():
    src = 'int a = 1;  // note\n/* block\n comment */ const char *s = "// kept /* too */";\nchar c = \'"\';\n'
    assert bench._code_tokens(src) == 'int a = 1; const char *s = "// kept /* too */"; char c = \'"\';'


def test_comment_edit_keeps_hash_code_edit_changes_it():
    base = "__global__ void k(float *x) {\n    x[0] = 1.0f;   // first\n}\n"
    comment = "__global__ void k(float *x) {\n    // a new remark\n    x[0] = 1.0f;   /* first */\n}\n"
    code = "__global__ void k(float *x) {\n    x[0] = 2.0f;   // first\n}\n"
    assert bench._code_tokens(base) == bench._code_tokens(comment)
    assert bench._code_tokens(base) != bench._code_tokens(code)
    assert bench._code_tokens('s = "a  b";') != bench._code_tokens('s = "a b";')  # inside a literal: code


def test_traffic_reported_only_for_matching_sources(tmp_path, monkeypatch):
    # a summary line names the hash of the sources its counters were taken with:
    # the figure is reported while the current sources hash the same, else null
    h = bench.kernel_source_hash()
    f = tmp_path / "counters.md"
    f.write_text("traffic: mg_smooth_level0 1234 bytes/launch sources %s\n"
                 "traffic: krylov_update 5678 bytes/launch sources 0000000000000000\n" % h)
    monkeypatch.setattr(bench, "COUNTERS", str(f))
    assert bench.measured_traffic("mg_smooth_level0") == 1234.0
    assert bench.measured_traffic("krylov_update") is None
    assert bench.measured_traffic("mac_saddle_apply") is None


def test_gpu_leg_loads_nothing_from_the_oracle():
    """Only the CPU-baseline leg (_cpu_step, run in worker processes) may import the
    oracle: the functions that build contexts and time the GPU reach the library
    through the binding alone, and no module-level import of bench reaches oracle/
    or the test helpers (which import the oracle)."""
    import ast
    import inspect
    tree = ast.parse(inspect.getsource(bench))
    users = set()
    for fn in [n for n in ast.walk(tree) if isinstance(n, (ast.FunctionDef, ast.ClassDef))]:
        for n in ast.walk(fn):
            mods = []
            if isinstance(n, ast.Import):
                mods = [a.name for a in n.names]
            elif isinstance(n, ast.ImportFrom):
                mods = [n.module or ""]
            if any(m.split(".")[0] in ("oracle", "tests") for m in mods):
                users.add(fn.name)
    assert users == {"_cpu_step"}, users
    top = [n for n in tree.body if isinstance(n, (ast.Import, ast.ImportFrom))]
    for n in top:
        names = [a.name for a in n.names] if isinstance(n, ast.Import) else [n.module or ""]
        assert not any(m.split(".")[0] in ("oracle", "tests") for m in names)
