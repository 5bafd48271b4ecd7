"""The packaged autotuner table (tuned_gfx950.txt beside libbm.so) is well formed: every
entry is "<shape class> | <configuration>" with the library's class key and a
configuration string of the specialised or generic kernel whose fields lie in the ranges
the library accepts (waves 1..8 per reference block, bounding-sweep row step 1..8,
candidate buffer 32..256 entries in multiples of 16)."""
import os
import re

TABLE = os.path.join(os.path.dirname(__file__), "..", "paper_2006_13714_amd", "tuned_gfx950.txt")
KEY = re.compile(r"^c(\d+) p(\d+) s(\d+) w(\d+) kr(\d+) prec([0-2]) hb(\d+) wb(\d+)$")
FAST = re.compile(r"^fast ws=(\d+) p1=(\d+) cap=(\d+)$")
GENERIC = re.compile(r"^generic wy=(\d+) wx=(\d+) cap=(\d+)$")


def entries():
    out = []
    for line in open(TABLE):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, sep, cfg = line.partition(" | ")
        assert sep, line
        out.append((key, cfg))
    return out


def test_every_entry_parses():
    es = entries()
    assert len(es) >= 100
    for key, cfg in es:
        m = KEY.match(key)
        assert m, key
        c, p, s, w, kr = (int(m.group(i)) for i in range(1, 6))
        assert 1 <= c <= 8 and 1 <= p <= 16 and s >= 1 and w >= 1 and kr in (1, 2, 4), key
        f = FAST.match(cfg)
        g = GENERIC.match(cfg)
        assert f or g, cfg
        if f:
            ws, p1, cap = (int(x) for x in f.groups())
            assert ws in (1, 2, 4, 8) and 1 <= p1 <= 8 and 32 <= cap <= 256 and cap % 16 == 0, cfg
        else:
            wy, wx, cap = (int(x) for x in g.groups())
            assert 1 <= wy * wx <= 4 and 32 <= cap <= 256 and cap % 16 == 0, cfg


def test_headline_classes_present():
    keys = {k for k, _ in entries()}
    # 512 x 512 gray, 8 x 8 patches, stride 3, 39 x 39 window, K = 16, each precision form;
    # the one-slab classes of the 3D workloads
    for prec in range(3):
        assert f"c1 p8 s3 w39 kr1 prec{prec} hb1 wb1" in keys
        assert f"c1 p6 s1 w30 kr1 prec{prec} hb1 wb1" in keys
        assert f"c3 p6 s1 w30 kr1 prec{prec} hb1 wb1" in keys
