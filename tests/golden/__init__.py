"""Fixtures of values the paper prints, each line citing the passage that prints it."""
import os

_HERE = os.path.dirname(os.path.abspath(__file__))


def printed(path="paper_printed_values.txt"):
    """Name -> (value, citation) from a fixture file of this folder."""
    out = {}
    with open(os.path.join(_HERE, path)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, value, cite = line.split(None, 2)
            out[name] = (float(value), cite)
    return out


def value(name):
    return printed()[name][0]
