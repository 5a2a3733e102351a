"""Reader of the `key = values` fixtures in this folder (comments after #)."""
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def read(name):
    out = {}
    with open(os.path.join(HERE, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, val = (s.strip() for s in line.split("=", 1))
            vals = [float(x) for x in val.split()]
            out[key] = vals if len(vals) > 1 else vals[0]
    return out
