"""Optional record of the parity errors the GPU tests measure: with the
environment variable LC_PARITY_LOG set to a path, each comparison appends one
JSON line (label, form, e_max, e_rms, compared cells)."""
import json
import os


def record(label, form, e_max, e_rms, cells=None):
    path = os.environ.get("LC_PARITY_LOG")
    if not path:
        return
    with open(path, "a") as f:
        f.write(json.dumps({"label": label, "form": form, "e_max": float(e_max), "e_rms": float(e_rms),
                            "cells": None if cells is None else int(cells)}) + "\n")
