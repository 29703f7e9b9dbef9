"""The tuner's table logic (CPU): the size classes, the per-class decision with its
margin and nearest-class fill, and the header it writes, which must reproduce the
committed pdt_tuning.h from that file's own table."""
import os
import re

from paper_2404_02844_amd import autotune

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TUNING = os.path.join(ROOT, "paper_2404_02844_amd", "csrc", "pdt_tuning.h")


def test_size_classes():
    assert [autotune.size_class(n) for n in (0, 1, 2, 3, 4, 255, 256, 257, 1 << 20)] == [0, 0, 1, 1, 2, 7, 8, 8, 15]


def test_decision_per_class():
    rows = [(0, 1, 5, 0, 16, 2.0, 1.0),      # class 4: eight waves twice as fast
            (0, 1, 5, 0, 256, 1.0, 0.97),    # class 8: inside the margin -> four
            (0, 1, 5, 0, 4096, 1.0, 1.5)]    # class 12: four faster
    t = autotune.decide(rows)[0][1][5]
    assert t[4] == 8 and t[8] == 4 and t[12] == 4
    # unmeasured classes take the nearest measured one (ties to the smaller)
    assert t[0] == 8 and t[5] == 8 and t[6] == 8 and t[7] == 4 and t[15] == 4
    # untouched entries stay four
    assert autotune.decide(rows)[1][0][3] == [4] * 16


def test_committed_header_is_the_tuner_format():
    text = open(TUNING).read()
    body = text[text.index("kKs[3][2][13][16] = {"):text.index("};")]
    nums = [int(x) for x in re.findall(r"\d+", body.split("=", 1)[1])]
    assert len(nums) == 3 * 2 * 13 * 16 and set(nums) <= {4, 8}
    table = [[[nums[((v * 2 + k) * 13 + nt) * 16:((v * 2 + k) * 13 + nt + 1) * 16] for nt in range(13)]
              for k in range(2)] for v in range(3)]
    assert autotune.header(table) == text
