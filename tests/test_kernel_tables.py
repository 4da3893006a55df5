"""The step kernel's packed per-link constants decode to the D2Q9 lattice the
paper prints (velocities of Sec. III and their opposites)."""
import json
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_packed_link_tables_match_paper():
    src = open(os.path.join(ROOT, "paper_1808_05168_amd", "csrc", "k_step.hip")).read()
    K = int(re.search(r"kCXp = (0x[0-9A-Fa-f]+)u", src).group(1), 16)
    Z = int(re.search(r"kCZp = (0x[0-9A-Fa-f]+)u", src).group(1), 16)
    O = int(re.search(r"kOppP = (0x[0-9A-Fa-f]+)ull", src).group(1), 16)
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_values.json")))
    c = gold["d2q9_velocities"]["c"]
    for l in range(9):
        assert ((K >> (2 * l)) & 3) - 1 == c[l][0]
        assert ((Z >> (2 * l)) & 3) - 1 == c[l][1]
        o = (O >> (4 * l)) & 15
        assert c[o] == [-c[l][0], -c[l][1]]
