"""Reader for the printed values in paper_values.txt."""
import os


def paper_values():
    out = {}
    with open(os.path.join(os.path.dirname(__file__), "paper_values.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            k, v = [x.strip() for x in line.split("=")]
            out[k] = float(v) if ("." in v or "e" in v) else int(v)
    return out
