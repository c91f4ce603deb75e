"""Host checks of the traffic-record helpers (no GPU needed)."""
import json

from paper_math_0610051_amd import pmc


def test_code_digest_ignores_comments_and_layout_only():
    base = 'int f(int x) {\n    return x + 1; // one\n}\nconst char *s = "a // b";\n'
    same = '/* header */\nint  f(int x)\n{ return x + 1;   }\n// trailing\nconst char *s = "a // b";'
    assert pmc._code_only(base) == pmc._code_only(same)
    # code inside string literals and a changed operator are code
    assert pmc._code_only(base) != pmc._code_only(base.replace('"a // b"', '"a /* b"'))
    assert pmc._code_only(base) != pmc._code_only(base.replace("x + 1", "x - 1"))
    # quotes inside comments do not open a literal
    assert pmc._code_only("int a; // it's\nint b;") == "int a; int b;"
    assert pmc._code_only("char q = '\"'; int c; /* \" */") == "char q = '\"'; int c;"


def test_traffic_record_is_rejected_when_stale(tmp_path):
    rec = {"kernel": "k_interp", "source_digest": pmc.source_digest(), "traffic_bytes": 1.0, "N": 1024}
    path = tmp_path / "rec.json"
    path.write_text(json.dumps(rec))
    assert pmc.load_traffic(str(path), "k_interp", N=1024) is not None
    assert pmc.load_traffic(str(path), "k_interp", N=512) is None
    assert pmc.load_traffic(str(path), "k_cols", N=1024) is None
    rec["source_digest"] = "0" * 64
    path.write_text(json.dumps(rec))
    assert pmc.load_traffic(str(path), "k_interp", N=1024) is None
    assert pmc.load_traffic(str(tmp_path / "missing.json"), "k_interp") is None


def test_traffic_file_holds_one_record_per_configuration(tmp_path):
    d = pmc.source_digest()
    recs = [{"kernel": "k_interp", "source_digest": d, "traffic_bytes": 1.0, "sigma": 2.0, "kernel_width": 5},
            {"kernel": "k_interp", "source_digest": d, "traffic_bytes": 2.0, "sigma": 1.5, "kernel_width": 6}]
    path = tmp_path / "recs.json"
    path.write_text(json.dumps({"records": recs}))
    assert pmc.load_traffic(str(path), "k_interp", sigma=2.0, kernel_width=5)["traffic_bytes"] == 1.0
    assert pmc.load_traffic(str(path), "k_interp", sigma=1.5, kernel_width=6)["traffic_bytes"] == 2.0
    assert pmc.load_traffic(str(path), "k_interp", sigma=1.75, kernel_width=6) is None
