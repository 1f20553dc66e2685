"""Writes worked_example.json.  Calls only the exact rational oracle.

The matrix is a hand-picked Hermitian positive-definite example with small
Gaussian-integer entries; the paper prints no numeric example, so every
stored value below is computed here in exact rational arithmetic and can be
re-checked by hand from the cofactor definitions (Eq. adjoint_elements) and
the real-part determinant (Eq. detr).
"""
import json
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
from oracle import exact  # noqa: E402

# a, d, f, Re b, Im b, Re c, Im c, Re e, Im e  for
# Z = [[4, 1+i, 2i], [1-i, 5, 1-i], [-2i, 1+i, 6]]
PACKED = [4, 5, 6, 1, 1, 0, 2, 1, -1]


def main():
    A = exact.unpack(PACKED)
    X, det = exact.inv_det(A)
    assert det.im == 0
    adj = [[x * det for x in row] for row in X]  # adjugate = det * inverse
    out = {
        "citation": "Section 2.1 (Eq. adjoint_elements: cofactors a_c..f_c), Section 3.1 "
                    "(Eq. inv_adjoint: A^-1 = adj/det; Eq. detr: real-part determinant)",
        "note": "Hand-checkable: a_c=df-|e|^2=28, b_c=c*conj(e)-b*f=-8-4i, c_c=b*e-c*d=2-10i, "
                "d_c=af-|c|^2=20, e_c=c*conj(b)-a*e=-2+6i, f_c=ad-|b|^2=18, "
                "det=a*a_c+Re(conj(b)b_c)+Re(conj(c)c_c)=112-12-20=80. "
                "Written by tests/golden/make_golden.py (exact rationals).",
        "packed_order": ["a", "d", "f", "Re b", "Im b", "Re c", "Im c", "Re e", "Im e"],
        "z": PACKED,
        "adjugate": [str(v) for v in exact.pack(adj)],
        "inverse": [str(v) for v in exact.pack(X)],
        "det": str(det.re),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "worked_example.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(path)


if __name__ == "__main__":
    main()
