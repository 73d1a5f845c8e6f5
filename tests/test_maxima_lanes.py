"""CPU check of the maxima pass's lane-to-column rule (csrc/nms_wave.h).

A wave covers a strip of 64 CW columns; lane l owns columns x0 + CW l ...
x0 + CW l + CW - 1.  A lane past the right edge loads the last CW columns
instead, and neighbouring lanes exchange their edge columns' vertical maxima
with wave shifts (lane l gets lane l - 1's last column as its left
neighbour and lane l + 1's first column, or column W - 1 when lane l + 1 is
past the edge, as its right neighbour); the strip's outer neighbours come
from two halo columns clamped into the image.  For the 3x3 window of
section 3's maxpool test to be right, the columns a valid column x sees
must be exactly the in-image members of {x - 1, x, x + 1}, possibly with
repeats of those members.  This emulates the index arithmetic for every
lane width and a range of widths."""
import pytest


def window_columns(W: int, CW: int):
    """{x: set of columns in x's horizontal window} as the wave computes it."""
    out = {}
    strips = (W + 64 * CW - 1) // (64 * CW)
    for s in range(strips):
        x0 = s * 64 * CW
        xl = [x0 + CW * l for l in range(64)]
        ok = [x < W for x in xl]
        xc = [xl[l] if ok[l] else W - CW for l in range(64)]
        cols = [[xc[l] + c for c in range(CW)] for l in range(64)]
        left_halo = min(max(x0 - 1, 0), W - 1)
        right_halo = min(max(x0 + 64 * CW, 0), W - 1)
        for l in range(64):
            if not ok[l]:
                continue
            left = cols[l - 1][CW - 1] if l > 0 else left_halo
            if l < 63:
                right = cols[l + 1][0] if ok[l + 1] else cols[l + 1][CW - 1]
            else:
                right = right_halo
            for c in range(CW):
                lft = cols[l][c - 1] if c > 0 else left
                rgt = cols[l][c + 1] if c + 1 < CW else right
                out[cols[l][c]] = {lft, cols[l][c], rgt}
    return out


@pytest.mark.parametrize("CW", [1, 2, 4])
def test_every_column_sees_its_in_image_neighbours(CW):
    for W in list(range(CW, 600, CW)) + [1020, 1024, 1028]:
        win = window_columns(W, CW)
        assert sorted(win) == list(range(W)), (W, CW)
        for x, seen in win.items():
            want = {c for c in (x - 1, x, x + 1) if 0 <= c < W}
            assert seen == want, (W, CW, x, seen, want)


def test_past_edge_lane_passes_the_last_column():
    """The case that a lane past the edge handing on its first column gets
    wrong: four columns per lane, W = 300, the last valid lane owns 296..299
    and must see 299 (not 296) to the right of 299."""
    assert window_columns(300, 4)[299] == {298, 299}
    assert window_columns(260, 4)[259] == {258, 259}
