"""Values the paper prints (paper_values.txt: key, value, citation per line)."""
import os

_HERE = os.path.dirname(os.path.abspath(__file__))


def _load():
    out = {}
    with open(os.path.join(_HERE, "paper_values.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, val, cite = line.split(None, 2)
            out[key] = (float(val), cite)
    return out


PAPER = _load()


def paper(key: str) -> float:
    """The printed value of key."""
    return PAPER[key][0]
