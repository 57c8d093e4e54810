"""Reader for the small hand-worked fixtures in tests/golden/.

Format: '#' comments; 'key: values' on one line; 'key:' followed by rows of
numbers until the next key; 'case: a b c | ... | ...' lines collected in a
list under 'case'.
"""
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _num(tok):
    if tok.lower().startswith(("0x", "-0x")):
        return int(tok, 16)
    try:
        return int(tok)
    except ValueError:
        return float(tok)


def load(name):
    out = {}
    key = None
    with open(os.path.join(GOLDEN, name)) as fh:
        for raw in fh:
            line = raw.split("#", 1)[0].strip()
            if not line:
                continue
            if ":" in line:
                k, v = line.split(":", 1)
                k, v = k.strip(), v.strip()
                if k == "case":
                    out.setdefault("case", []).append(
                        [[_num(t) for t in part.split()] for part in v.split("|")])
                    key = None
                elif v:
                    vals = [_num(t) for t in v.split()]
                    out[k] = vals[0] if len(vals) == 1 else vals
                    key = None
                else:
                    key = k
                    out[k] = []
            elif key is not None:
                out[key].append([_num(t) for t in line.split()])
    return out
