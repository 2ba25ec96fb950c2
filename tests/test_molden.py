"""CPU tests of the .molden geometry reader and writer (host I/O)."""
import numpy as np

from paper_2510_25938_amd.molden import BOHR_TO_ANGSTROM, read_first_geometry, write_geometries


def test_atoms_section_round_trip(tmp_path):
    p = tmp_path / "in.molden"
    p.write_text("[Molden Format]\n[Atoms] Angs\nAr 1 18 0.0 0.0 0.0\nAr 2 18 1.1225 0.0 0.0\n"
                 "Ar 3 18 0.5 0.9 0.1\n[GTO]\n")
    flat, syms = read_first_geometry(str(p))
    assert syms == ["Ar"] * 3
    assert np.allclose(flat, [0, 0, 0, 1.1225, 0, 0, 0.5, 0.9, 0.1])
    q = tmp_path / "out.molden"
    write_geometries(str(q), [flat, flat * 2], [-3.0, -1.5], syms)
    back, s2 = read_first_geometry(str(q))
    assert s2 == syms and np.allclose(back, flat)
    assert q.read_text().count("E = ") == 2


def test_atoms_in_bohr_are_converted(tmp_path):
    p = tmp_path / "au.molden"
    p.write_text("[Molden Format]\n[Atoms] AU\nX 1 0 1.0 2.0 3.0\n")
    flat, _ = read_first_geometry(str(p))
    assert np.allclose(flat, np.array([1.0, 2.0, 3.0]) * BOHR_TO_ANGSTROM)


def test_first_frame_of_geometries(tmp_path):
    p = tmp_path / "g.molden"
    p.write_text("[Molden Format]\n[GEOMETRIES] XYZ\n 2\n first\nAr 0 0 0\nAr 0 0 1.5\n"
                 " 2\n second\nAr 0 0 0\nAr 0 0 9.0\n")
    flat, syms = read_first_geometry(str(p))
    assert np.allclose(flat, [0, 0, 0, 0, 0, 1.5]) and syms == ["Ar", "Ar"]
