"""Host logic of bench.py that needs no GPU: the code hash that keys the
committed counter records (traffic per launch) to the sources they were
taken from."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_code_text_drops_comments_only():
    a = 'int x = 1; // one\n/* two\n lines */ const char *s = "a // b /* c */";\nchar q = \'"\';\n'
    b = 'int x = 1;\n   const char *s = "a // b /* c */"; // other\nchar q = \'"\'; /* x */\n'
    c = 'int x = 2; // one\n/* two\n lines */ const char *s = "a // b /* c */";\nchar q = \'"\';\n'
    d = 'int x = 1; // one\n/* two\n lines */ const char *s = "a // b  /* c */";\nchar q = \'"\';\n'
    # white space is collapsed outside literals (literals stand apart)
    assert bench.code_text(a) == 'int x = 1; const char *s = "a // b /* c */" ; char q = \'"\' ;'
    assert bench.code_text(a) == bench.code_text(b)
    assert bench.code_text(a) != bench.code_text(c)      # a changed constant
    assert bench.code_text(a) != bench.code_text(d)      # a changed string literal


def test_counter_records_name_existing_sources():
    with open(bench.TRAFFIC_FILE) as f:
        recs = json.load(f)
    assert recs
    for key, rec in recs.items():
        assert len(key.split(":")) == 3, key
        for rel in rec["sources"]:
            assert os.path.isfile(os.path.join(ROOT, rel)), (key, rel)
        assert os.path.isfile(os.path.join(ROOT, rec["profile"])), key
        assert rec["bytes_per_launch"] > rec["algorithmic_bytes"] > 0, key


def test_more_than_one_gpu_is_refused():
    """The engine runs on one GPU: asking bench.py for more exits with a
    message (before any GPU work), also under a launcher's WORLD_SIZE."""
    import subprocess
    env = dict(os.environ)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 2 and "one GPU" in r.stderr, (r.returncode, r.stderr)
    env["WORLD_SIZE"] = "4"
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")],
                       capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 2 and "one GPU" in r.stderr, (r.returncode, r.stderr)
