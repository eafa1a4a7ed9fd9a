"""Writes contact_values.json: eq (Cij) of the paper, C(r) = (1-(r/r0)^6)/(1-(r/r0)^10),
evaluated in exact rational arithmetic at r0 = 7.5 A (the paper's typical reference
distance) for a handful of distances, then rounded once to double.  r = r0 uses the
limit 3/5 of the removable singularity."""
import json
import os
from fractions import Fraction as F

R0 = F(15, 2)
RS = ["0.5", "3.8", "4.0", "6.0", "7.5", "9.0", "10.0", "12.0", "15.0", "30.0"]


def C(r):
    u = r / R0
    if u == 1:
        return F(3, 5)
    return (1 - u ** 6) / (1 - u ** 10)


vals = [[float(F(s)), float(C(F(s)))] for s in RS]
out = {"source": "eq (Cij), exact rational evaluation", "r0": 7.5, "values": vals}
with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "contact_values.json"), "w") as f:
    json.dump(out, f, indent=1)
