"""Writes hand_cases.json: small meshes whose intersection status follows from
their construction (stated in each case's "why").  No oracle or library
call is made; the expected values are geometric facts about exact dyadic
coordinates.  Semantics: closed surfaces, touching counts (the reading of
Section 3.2's overlap predicate for closed sets; Section 3.6 discusses the
contact cases).  Each case also states whether A contains B or lies within
B with no shared surface point (the containment join of Section 3.3 and its
inverse), the facts the containment predicates are checked against.

Run:  python tests/golden/make_hand_cases.py
"""
import json
import os

import numpy as np

TET_V = [[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]]
TET_F = [[0, 2, 1], [0, 1, 3], [0, 3, 2], [1, 2, 3]]
OCT_V = [[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]]
OCT_F = [[0, 2, 4], [2, 1, 4], [1, 3, 4], [3, 0, 4], [2, 0, 5], [1, 2, 5], [3, 1, 5], [0, 3, 5]]
CUBE_V = [[x, y, z] for x in (0, 1) for y in (0, 1) for z in (0, 1)]
CUBE_F = [[0, 1, 3], [0, 3, 2], [4, 6, 7], [4, 7, 5], [0, 4, 5], [0, 5, 1],
          [2, 3, 7], [2, 7, 6], [0, 2, 6], [0, 6, 4], [1, 5, 7], [1, 7, 3]]


def box(lo, hi):
    return [[(lo[0], hi[0])[i], (lo[1], hi[1])[j], (lo[2], hi[2])[k]]
            for i in (0, 1) for j in (0, 1) for k in (0, 1)]


def tr(v, d):
    return [[a + b for a, b in zip(p, d)] for p in v]


def sc(v, s):
    return [[a * s for a in p] for p in v]


ULP1 = float(np.nextafter(np.float32(1.0), np.float32(2.0)))  # 1 + 2^-23
D12 = 2.0 ** -12

CASES = [
    ("vertex_vertex", TET_V, TET_F, tr(TET_V, [1, 0, 0]), TET_F, True,
     "A={x,y,z>=0,x+y+z<=1}; B=A+(1,0,0) has x>=1; the only common point is (1,0,0), a vertex of both"),
    ("vertex_on_face", TET_V, TET_F,
     [[0.25, 0.25, 0.5], [1, 1, 1], [2, 1, 1], [1, 2, 1]], [[0, 1, 2], [0, 2, 3], [0, 3, 1], [1, 3, 2]], True,
     "B lies in x+y+z>=1 and meets that plane only at its vertex (1/4,1/4,1/2), interior to A's face x+y+z=1"),
    ("vertex_on_edge", TET_V, TET_F,
     [[0.5, 0.5, 0], [2, 2, -1], [3, 2, -1], [2, 3, -1]], [[0, 1, 2], [0, 2, 3], [0, 3, 1], [1, 3, 2]], True,
     "B lies in z<=0 and x+y+z>=1, A in z>=0 and x+y+z<=1; they share only B's vertex (1/2,1/2,0), on A's edge (1,0,0)-(0,1,0)"),
    ("edge_edge", TET_V, TET_F,
     [[0.5, 0.5, -1], [0.5, 0.5, 1], [2, 1, 0], [1, 2, 0.5]], [[0, 1, 2], [0, 2, 3], [0, 3, 1], [1, 3, 2]], True,
     "B lies in x+y>=1 and touches that plane along its edge x=y=1/2; A meets x+y=1 only on its edge (1,0,0)-(0,1,0); the edges cross at (1/2,1/2,0)"),
    ("coplanar_overlap", TET_V, TET_F,
     [[0.25, 0.25, 0], [1.25, 0.25, 0], [0.25, 1.25, 0], [0.25, 0.25, -1]], [[0, 1, 2], [0, 3, 1], [0, 2, 3], [1, 3, 2]], True,
     "A in z>=0, B in z<=0; their faces in z=0 overlap in an area"),
    ("coplanar_shared_edge", TET_V, TET_F,
     [[1, 0, 0], [0, 1, 0], [1, 1, 0], [0.5, 0.5, -1]], [[0, 2, 1], [0, 1, 3], [1, 2, 3], [2, 0, 3]], True,
     "A in z>=0, B in z<=0; in z=0 A's face and B's face share exactly the edge (1,0,0)-(0,1,0)"),
    ("disjoint_2e-12", TET_V, TET_F, tr(TET_V, [1 + D12, 0, 0]), TET_F, False,
     "B has x>=1+2^-12 while A has x<=1"),
    ("coplanar_gap_2e-12", TET_V, TET_F,
     [[1 + D12, 0, 0], [D12, 1, 0], [1 + D12, 1, 0], [0.5, 0.5, -1]], [[0, 2, 1], [0, 1, 3], [1, 2, 3], [2, 0, 3]], False,
     "in z=0, B's face has x+y>=1+2^-12 while A has x+y<=1; off that plane A and B are on opposite sides"),
    ("nested_octahedra", OCT_V, OCT_F, sc(OCT_V, 0.5), OCT_F, False,
     "B={|x|+|y|+|z|<=1/2} lies strictly inside A={|x|+|y|+|z|<=1}: the surfaces never meet"),
    ("crossing", TET_V, TET_F, tr(TET_V, [0.25, 0.25, 0.25]), TET_F, True,
     "B's vertex (1/4,1/4,1/4) is inside A and B's vertex (5/4,1/4,1/4) outside, so B's surface crosses A's"),
    ("identical", OCT_V, OCT_F, OCT_V, OCT_F, True, "same surface"),
    ("cube_face_contact", CUBE_V, CUBE_F, tr(CUBE_V, [1, 0.5, 0.25]), CUBE_F, True,
     "A=[0,1]^3, B=[1,2]x[1/2,3/2]x[1/4,5/4]: the faces in x=1 overlap"),
    ("cube_face_gap_1ulp", CUBE_V, CUBE_F, box([ULP1, 0.5, 0.25], [2, 1.5, 1.25]), CUBE_F, False,
     "B has x>=1+2^-23 (one FP32 ulp above 1) while A has x<=1"),
    ("cube_nested", CUBE_V, CUBE_F, tr(sc(CUBE_V, 0.5), [0.25, 0.25, 0.25]), CUBE_F, False,
     "B=[1/4,3/4]^3 strictly inside A=[0,1]^3"),
    ("cube_poke_through", CUBE_V, CUBE_F, tr(sc(CUBE_V, 0.5), [0.75, 0.25, 0.25]), CUBE_F, True,
     "B=[3/4,5/4]x[1/4,3/4]^2 crosses A's face x=1"),
    ("cube_edge_contact", CUBE_V, CUBE_F, tr(CUBE_V, [1, 1, 0.5]), CUBE_F, True,
     "B=[1,2]x[1,2]x[1/2,3/2] meets A=[0,1]^3 along the segment x=y=1, z in [1/2,1]"),
    ("cube_corner_contact", CUBE_V, CUBE_F, tr(CUBE_V, [1, 1, 1]), CUBE_F, True,
     "B=[1,2]^3 meets A=[0,1]^3 only at the corner (1,1,1)"),
    ("nested_octahedra_reversed", sc(OCT_V, 0.5), OCT_F, OCT_V, OCT_F, False,
     "A={|x|+|y|+|z|<=1/2} lies strictly inside B={|x|+|y|+|z|<=1}"),
    ("cube_nested_corner_touch", CUBE_V, CUBE_F, sc(CUBE_V, 0.5), CUBE_F, True,
     "B=[0,1/2]^3 inside A=[0,1]^3 shares A's corner region: the faces x=0, y=0, z=0 of both overlap"),
    ("cube_nested_offcentre", CUBE_V, CUBE_F, tr(sc(CUBE_V, 0.25), [0.5, 0.125, 0.625]), CUBE_F, False,
     "B=[1/2,3/4]x[1/8,3/8]x[5/8,7/8] strictly inside A=[0,1]^3"),
    ("octahedron_in_cube", box([-2, -2, -2], [2, 2, 2]), CUBE_F, OCT_V, OCT_F, False,
     "B={|x|+|y|+|z|<=1} strictly inside A=[-2,2]^3"),
]

# containment facts: (A contains B, A within B) with no shared surface point
INSIDE = {
    "nested_octahedra": (True, False),
    "cube_nested": (True, False),
    "nested_octahedra_reversed": (False, True),
    "cube_nested_offcentre": (True, False),
    "octahedron_in_cube": (True, False),
}


def main():
    out = []
    for name, va, fa, vb, fb, exp, why in CASES:
        for v in (va, vb):
            a = np.asarray(v, np.float64)
            assert np.all(a.astype(np.float32).astype(np.float64) == a), name  # exact in FP32
        contains, within = INSIDE.get(name, (False, False))
        assert not (exp and (contains or within)), name  # a shared point excludes containment
        out.append(dict(name=name, expected=bool(exp), contains=contains, within=within, why=why,
                        A=dict(verts=va, faces=fa), B=dict(verts=vb, faces=fb)))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "hand_cases.json")
    with open(path, "w") as fh:
        json.dump(dict(source="constructed; expected values follow from each 'why'", cases=out), fh, indent=1)
    print("wrote", path, len(out), "cases")


if __name__ == "__main__":
    main()
