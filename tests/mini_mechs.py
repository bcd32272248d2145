"""Hand-built tiny mechanisms with closed-form behaviour (test inputs only)."""
import numpy as np

from paper_2011_07978_amd.synth import Mechanism

P_ATM = 1.01325e6
RU_ERG = 8.314462618e7


def isomerisation(A=1e6, delta_a7=0.0, third_body=False, eff=None, b=0.0, Ea=0.0):
    """A <=> B between two isomers (same atoms, same molar mass, same a1..a6).

    Then the reaction enthalpy is zero (dT/dt = 0), the mean molar mass is
    constant, sum(nu) = 0 and ln Kc = a7_B - a7_A, so dY_A/dt = -k Y_A + k' Y_B
    is linear with k = A T^b exp(-Ea/RT) (times [M] for a third-body reaction)
    and k' = k exp(-(a7_B - a7_A)).  Species 2 is a non-reacting diluent.
    """
    comp = np.array([[1, 1, 0], [1, 1, 0], [0, 0, 2]], np.int32)
    em = np.array([1.008, 12.011, 15.999])
    W = (comp * em).sum(1).astype(float)
    nasa = np.zeros((3, 7))
    nasa[:, 0] = 3.5
    nasa[:, 1] = 1e-4
    nasa[:, 5] = -1000.0
    nasa[0, 6] = 5.0
    nasa[1, 6] = 5.0 + delta_a7
    nasa[2, 6] = 4.0
    er, es, ev = [], [], []
    if eff:
        for s, v in eff.items():
            er.append(0); es.append(s); ev.append(v)
    return Mechanism(3, 3, 1, em, comp, W, nasa,
                     np.array([[0, -1]], np.int32), np.array([[1, -1, -1]], np.int32),
                     np.array([A]), np.array([b]), np.array([Ea]),
                     np.array([1 if third_body else 0], np.int32),
                     np.array(er, np.int32), np.array(es, np.int32), np.array(ev, float),
                     name="isomerisation")
