""".molden geometry I/O (Methodology, "Initial Structures and Input"; Running the Code).

read_first_geometry: the first geometry of a .molden file, from its [Atoms]
section or, failing that, the first frame of a [GEOMETRIES] XYZ section.
Returned as the paper's flattened [x0, y0, z0, x1, ...] array plus symbols.
write_geometries: a multi-frame [GEOMETRIES] XYZ file (one frame per accepted
structure, energy in the comment line), as the paper's *_accepted.molden.
Coordinates are taken as reduced LJ units (sigma = 1) unless scaled by the caller.
"""
import numpy as np

BOHR_TO_ANGSTROM = 0.529177210903


def _sections(lines):
    out, name, start = {}, None, 0
    for i, ln in enumerate(lines):
        s = ln.strip()
        if s.startswith("[") and "]" in s:
            if name is not None:
                out.setdefault(name, (start, i, header))
            name = s[1:s.index("]")].strip().lower()
            header = s[s.index("]") + 1:].strip().lower()
            start = i + 1
    if name is not None:
        out.setdefault(name, (start, len(lines), header))
    return out


def read_first_geometry(path):
    """(flat coordinates float64 [3N], symbols list) of the first geometry."""
    with open(path) as fh:
        lines = fh.read().splitlines()
    secs = _sections(lines)
    if "atoms" in secs:
        a, b, unit = secs["atoms"]
        syms, xyz = [], []
        for ln in lines[a:b]:
            f = ln.split()
            if len(f) >= 6:
                syms.append(f[0])
                xyz.append([float(v) for v in f[3:6]])
        if syms:
            arr = np.array(xyz, dtype=np.float64)
            if unit.startswith("au") or unit.startswith("bohr"):
                arr *= BOHR_TO_ANGSTROM
            return arr.reshape(-1), syms
    if "geometries" in secs:
        a, b, _ = secs["geometries"]
        body = [ln for ln in lines[a:b]]
        i = 0
        while i < len(body) and not body[i].strip():
            i += 1
        n = int(body[i].split()[0])
        syms, xyz = [], []
        for ln in body[i + 2:i + 2 + n]:
            f = ln.split()
            syms.append(f[0])
            xyz.append([float(v) for v in f[1:4]])
        return np.array(xyz, dtype=np.float64).reshape(-1), syms
    raise ValueError(f"{path}: no [Atoms] or [GEOMETRIES] XYZ section")


def write_geometries(path, frames, energies, symbols):
    """Write frames ([3N] flat arrays) as a multi-frame [GEOMETRIES] XYZ file."""
    with open(path, "w") as fh:
        fh.write("[Molden Format]\n[GEOMETRIES] XYZ\n")
        for flat, e in zip(frames, energies):
            xyz = np.asarray(flat, dtype=np.float64).reshape(-1, 3)
            fh.write(f"{len(xyz):6d}\n E = {e:.10f}\n")
            for s, (x, y, z) in zip(symbols, xyz):
                fh.write(f" {s:<3s} {x:18.10f} {y:18.10f} {z:18.10f}\n")
