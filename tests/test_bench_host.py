"""Host logic of bench.py: the D(t) error against the oracle reported in its
JSON line, and the refusal of more than one GPU. No GPU."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_d_error_vs_oracle():
    t = np.arange(50)
    D_ref = np.stack([bench.D_B * np.exp(-t / 10.0), bench.D_B * np.ones(50), np.zeros(50)])
    e = bench.d_error_vs_oracle(D_ref.copy(), D_ref)
    assert e["max_rel"] == 0.0 and e["times"] == 50 and e["directions"] == 3 and e["tolerance"] == 1e-5
    D = D_ref.copy()
    D[1, 7] *= 1 + 3e-6                                   # relative to D itself
    assert np.isclose(bench.d_error_vs_oracle(D, D_ref)["max_rel"], 3e-6)
    D = D_ref.copy()
    D[2, 3] = 1e-9                                       # D_ref = 0: the floor 1e-2 D_b applies
    assert np.isclose(bench.d_error_vs_oracle(D, D_ref)["max_rel"], 1e-9 / (1e-2 * bench.D_B))


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0 and "one GPU" in r.stderr and r.stdout == ""


def test_traffic_key_ignores_comments_only():
    """The traffic record's key: a comment or blank-line edit keeps it, a code
    edit changes it; literals that look like comments are code."""
    import hashlib
    import bench
    a = 'int f() { return 1; } // one\nconst char* s = "a//b /* c */";\n'
    b = '/* header */\n  int f() { return 1; }\n\n  const char* s = "a//b /* c */"; // two\n'
    c = 'int f() { return 2; }\nconst char* s = "a//b /* c */";\n'
    h = lambda s: hashlib.sha256(bench.strip_comments(s).encode()).hexdigest()
    assert bench.strip_comments(a) == 'int f() { return 1; }\nconst char* s = "a//b /* c */";'
    assert h(a) != h(c)
    assert h(b) == h(a)
