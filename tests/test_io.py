"""CPU checks of the file formats of the library (no GPU needed): the OFF
reader with per-face radius indices (Section 6 of the paper) and the CSV
readers of particle states and contact springs."""
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def sdem():
    from paper_2507_12610_amd import sdem as S
    if not os.path.exists(S.LIB_PATH):
        pytest.skip("libsdem.so not built")
    return S


OFF_TEXT = """# a mesh of every kind of face
OFF
5 5 0
0 0 0
1 0 0
1 1 0
0 1 0   # vertex 3
0.5 0.5 2.0

4 0 1 2 3        # rectangle, default radius index
3 0 1 4 2        # triangle with radius index 2
2 3 4 1          # segment with radius index 1
1 4 1 0.5 0.5 0.5  # point: radius index, then colour values
3 1 2 4
"""


def test_off_faces_of_every_kind(sdem, tmp_path):
    p = tmp_path / "mesh.off"
    p.write_text(OFF_TEXT)
    els, rm = sdem.read_off(str(p), radii=[0.002, 0.02, 0.01])
    assert [len(e) for e in els] == [4, 3, 2, 1, 3]
    V = np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0], [0.5, 0.5, 2.0]], float)
    assert np.array_equal(els[0], V[[0, 1, 2, 3]])
    assert np.array_equal(els[1], V[[0, 1, 4]])
    assert np.array_equal(els[2], V[[3, 4]])
    assert np.array_equal(els[3], V[[4]])
    assert np.array_equal(rm, [0.002, 0.01, 0.02, 0.02, 0.002])


@pytest.mark.parametrize("bad,word", [
    ("OFF\n2 1 0\n0 0 0\n1 0 0\n5 0 1 0 1 0\n", "1 to 4"),
    ("OFF\n2 1 0\n0 0 0\n1 0 0\n2 0 7\n", "out of range"),
    ("OFF\n2 1 0\n0 0 0\n1 0 0\n2 0 1 3\n", "radius index"),
    ("OFF\n2 1 0\n0 0 0\n1 0 nan\n2 0 1\n", "bad vertex"),
    ("OFF\n3 1 0\n0 0 0\n1 0 0\n", "missing"),
    ("PLY\n", "no OFF header"),
])
def test_off_errors(sdem, tmp_path, bad, word):
    p = tmp_path / "bad.off"
    p.write_text(bad)
    with pytest.raises(sdem.SdemError) as ei:
        sdem.read_off(str(p), radii=[0.0, 1e-3])
    assert word in str(ei.value)


def test_csv_columns_by_name_and_ids(sdem, tmp_path):
    p = tmp_path / "in.csv"
    p.write_text("R, z, y, x, id, vx\n"
                 "0.002, 3, 2, 1, 1, 0.5\n"
                 "0.003, 6, 5, 4, 0, -0.5\n")
    st = sdem.read_csv(str(p))
    assert np.array_equal(st["x"], [[4, 5, 6], [1, 2, 3]])
    assert np.array_equal(st["R"], [0.003, 0.002])
    assert np.array_equal(st["v"], [[-0.5, 0, 0], [0.5, 0, 0]])
    assert np.array_equal(st["w"], np.zeros((2, 3)))
    assert np.array_equal(st["q"], [[1, 0, 0, 0], [1, 0, 0, 0]])


def test_csv_round_trip_digits(sdem, tmp_path):
    """17 significant digits read back to the same doubles."""
    rng = np.random.default_rng(0)
    x = rng.normal(size=(50, 3)) * 1e-3
    R = rng.uniform(1e-4, 1e-3, 50)
    p = tmp_path / "rt.csv"
    with open(p, "w") as f:
        f.write("x,y,z,R\n")
        for a, r in zip(x, R):
            f.write("%.17g,%.17g,%.17g,%.17g\n" % (*a, r))
    st = sdem.read_csv(str(p))
    assert np.array_equal(st["x"], x) and np.array_equal(st["R"], R)


@pytest.mark.parametrize("bad,word", [
    ("x,y,R\n1,2,3\n", "column z"),
    ("x,y,z,R\n1,2,3,0\n", "radius"),
    ("x,y,z,R,id\n1,2,3,1,0\n1,2,3,1,0\n", "permutation"),
    ("x,y,z,R\n1,2,abc,1\n", "bad value"),
])
def test_csv_errors(sdem, tmp_path, bad, word):
    p = tmp_path / "bad.csv"
    p.write_text(bad)
    with pytest.raises(sdem.SdemError) as ei:
        sdem.read_csv(str(p))
    assert word in str(ei.value)


def test_contacts_csv(sdem, tmp_path):
    p = tmp_path / "c.csv"
    p.write_text("ki,kj,usx,usy,usz,urx,ury,urz,ut\n"
                 "0,1,1e-6,0,0,0,2e-7,0,3e-8\n"
                 "2,-4,0,0,0,0,0,0,-1e-9\n")
    c = sdem.read_contacts_csv(str(p))
    assert c["ki"].tolist() == [0, 2] and c["kj"].tolist() == [1, -4]
    assert np.array_equal(c["us"][0], [1e-6, 0, 0]) and c["ut"][1] == -1e-9
