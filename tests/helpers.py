"""Shared test helpers: key material and encryptions drawn from the seeded
generator and built by the oracle (test infrastructure only)."""
import numpy as np

import oracle
import synth


class Keys:
    def __init__(self, P, seed, rot_ks=(), conj=False):
        self.P = P
        self.s = synth.stream(seed, "secret").ternary(P.n, 64)
        mods = P.q + P.p
        st = synth.stream(seed, "rlk")
        self.rlk = oracle.relin_key(P, self.s, np.stack([st.residues(mods, P.n) for _ in range(P.dnum)]),
                                    np.stack([st.gaussian(P.n) for _ in range(P.dnum)]))
        self.rot = {}
        for k in rot_ks:
            st = synth.stream(seed, "rot/%d" % k)
            self.rot[k] = oracle.rotation_key(P, self.s, k, np.stack([st.residues(mods, P.n) for _ in range(P.dnum)]),
                                              np.stack([st.gaussian(P.n) for _ in range(P.dnum)]))
        self.conj = None
        if conj:
            st = synth.stream(seed, "conj")
            self.conj = oracle.conj_key(P, self.s, np.stack([st.residues(mods, P.n) for _ in range(P.dnum)]),
                                        np.stack([st.gaussian(P.n) for _ in range(P.dnum)]))

    def encrypt(self, z, scale, level, name):
        P = self.P
        st = synth.stream(0, "enc/" + name)
        return oracle.encrypt(P, oracle.encode(z, P.log_n, scale), self.s, level,
                              st.residues(P.q[:level], P.n), st.gaussian(P.n))
