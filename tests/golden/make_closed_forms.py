"""Writes closed_forms.txt: LDP codes of small images derived in closed form.

The expected codes come from the definition worked by hand (Eqs. 1-3 with the
Kirsch compass masks); this script only formats them and calls nothing else.
Run: python tests/golden/make_closed_forms.py
"""
import os

RING = [(0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1), (1, 0), (1, 1)]
NAMES = ["E", "NE", "N", "NW", "W", "SW", "S", "SE"]


def rotl8(c, s):
    return ((c << s) | (c >> (8 - s))) & 255


def main():
    L = [
        "# Closed-form LDP codes derived by hand from the definition (Eqs. 1-3, Sections 2.2.1-2.2.2)",
        "# with the Kirsch compass masks M0..M7 = E, NE, N, NW, W, SW, S, SE (Fig. 1).",
        "# Each mask weighs its three ring neighbours centred on its direction with +5, the other five",
        "# with -3 and the centre with 0, so m_i = 8*S_i - 3*T (S_i: sum of mask i's +5 triple, T: sum",
        "# of the 8 neighbours).  Format: 'case NAME', 'k K', 'why TEXT', 'image H W' + H rows,",
        "# 'codes h w' + h rows (interior code map).  Written by make_closed_forms.py.",
    ]
    for j, (dx, dy) in enumerate(RING):
        trip = "%d,%d,%d" % ((j - 1) % 8, j, (j + 1) % 8)
        for k in (2, 3, 4):
            L.append("case impulse_%s_k%d" % (NAMES[j], k))
            L.append("k %d" % k)
            if k < 4:
                why = ("value 200 at ring neighbour %s only: masks %s respond +1000, the other five -600; "
                       "the k-th largest is +1000 and all three tied responses reach it (Eq. 3 uses >=), "
                       "so bits %s are set" % (NAMES[j], trip, trip))
                exp = rotl8(131, j)
            else:
                why = ("value 200 at ring neighbour %s only: masks %s respond +1000, the other five -600; "
                       "the 4th largest is -600, every response reaches it, all bits are set" % (NAMES[j], trip))
                exp = 255
            L.append("why " + why)
            L.append("image 3 3")
            img = [[0] * 3 for _ in range(3)]
            img[1 + dx][1 + dy] = 200
            L.extend(" ".join(map(str, r)) for r in img)
            L.append("codes 1 1")
            L.append(str(exp))
        L.append("case hole_%s_k3" % NAMES[j])
        L.append("k 3")
        L.append("why all 255 except 0 at ring neighbour %s: masks %s respond -1275, the five others tie "
                 "at +765; all five reach the 3rd largest (Eq. 3 uses >=), so five bits are set, the "
                 "complement of the impulse code" % (NAMES[j], trip))
        L.append("image 3 3")
        img = [[255] * 3 for _ in range(3)]
        img[1 + dx][1 + dy] = 0
        L.extend(" ".join(map(str, r)) for r in img)
        L.append("codes 1 1")
        L.append(str((~rotl8(131, j)) & 255))
    L.append("case vertical_step_k3")
    L.append("k 3")
    L.append("why columns 3-5 are 255, columns 0-2 are 0: columns 1 and 4 see a flat neighbourhood (all "
             "eight responses 0, code 255); at columns 2 and 3 the three largest responses are E, NE, SE "
             "(3825/1785/1785 and 2295/2295/2295)")
    L.append("image 5 6")
    L.extend("0 0 0 255 255 255" for _ in range(5))
    L.append("codes 3 4")
    L.extend("255 131 131 255" for _ in range(3))
    for k in range(1, 9):
        L.append("case flat_k%d" % k)
        L.append("k %d" % k)
        L.append("why a constant image makes all eight responses 0; every one equals the k-th largest, "
                 "so all bits are set for every k")
        L.append("image 4 5")
        L.extend("77 77 77 77 77" for _ in range(4))
        L.append("codes 2 3")
        L.extend("255 255 255" for _ in range(2))
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "closed_forms.txt")
    with open(out, "w") as f:
        f.write("\n".join(L) + "\n")


if __name__ == "__main__":
    main()
