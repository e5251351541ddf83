// One environment of a mobile-manipulator plan (device function).
//
// pick-and-place (Sec. IV-A, pi_p&p without the final move to Exit):
//   move_to(x, y, psi, v) -> grasp(q) -> move_to(x, y, psi, v) -> place(x, y, z, psi)
// move-and-push (Sec. IV-A, pi_m&p):
//   move_to(x, y, psi, v) -> push(start xyz, heading, distance, speed,
//   approach height, gripper yaw): closed fingers reach a pose above the start
//   point, descend to it, sweep the end effector along the push line, then
//   the gripper opens.
// Problem 2 cost: dt per control step while the active action is not yet
// successful; tier 0 if every action succeeded and psi_g holds at T (the
// object rests on the goal table's top face, or with its centre inside the
// goal box), 1 if every action succeeded but psi_g fails, 2 otherwise, 3
// diverged.  The object's contacts use its per-instance friction draw when
// the scene has one.
//
// Each action runs from the step after the previous one ends (Problem 1,
// t_{0,i+1} = T_i + 1) until success or timeout.  Controllers: straight-line
// base reference at the commanded speed (smoothstep-timed) tracked by joint
// PD, arm joint targets from damped-least-squares IK solved on the GPU at
// action start and tracked along smoothstep joint-space blends, finger PD;
// torques clamped to inom * accel_max.
//
// Dynamics per substep: Featherstone's articulated-body algorithm in three
// passes over the fixed 11-body tree (base x, base y, base yaw, six arm
// joints, two fingers on the last arm body).  Each pass runs one loop per
// segment of the tree (the chain, then the fingers off the palm), so no body
// selects its parent's data.  The contact forces on the base and finger links
// are taken off their bias forces between the first and second passes, and
// the semi-implicit Euler update is folded into the last; the object is a
// free box against the ground, the static boxes and the fingers (vertex-face
// both ways, one pass per contact of a lane).
//
// One environment per lane.  The per-body quantities the three passes hand to
// each other (joint state, bias accelerations, bias forces / U columns, D^-1,
// u) and the push's third joint-space anchor live in LDS, one lane-contiguous
// row per quantity, so the passes loop over bodies without unrolling and
// without scratch; the rest of the state stays in VGPRs.  HBM is touched only
// for z in and (cost, tier, pose) out; the scene is read through wave-uniform
// scalar loads.
#pragma once
#include "robot_spec.hpp"

namespace cem {
namespace {

constexpr int PP_LANES = 64;  // lanes sharing one LDS block of rows
// LDS rows (each PP_LANES floats):
//   q, qd (11 each); qref (10: joints 0..8, one row for both fingers);
//   the bias accelerations c_j = v_j x (S_j qd_j) that are not identically zero:
//     bodies 0, 1 only translate, so c_0 = c_1 = 0; body 2's angular velocity
//     is its own joint's, so c_2 has a zero angular part; the fingers slide,
//     so theirs is zero too: 3 rows for body 2, 6 for each of bodies 3..8, 3
//     for each finger (45);
//   the bias force pA (pass 1), then U / D (passes 2, 3) (6 per body);
//   u / D (11).
// 154 rows x 256 B = 39,424 B per wave: four waves fit in a CU's LDS.
constexpr int R_Q = 0, R_QD = R_Q + NJ, R_QREF = R_QD + NJ, R_C = R_QREF + PALM + 2, R_P = R_C + 3 + 6 * NARM + 6,
              R_UD = R_P + 6 * NJ, R_ROWS = R_UD + NJ;
static_assert(R_ROWS * PP_LANES * 4 <= 40960, "four waves per CU");

struct Lds {
  float *m;
  int lane;
  __device__ __forceinline__ float &at(int row) const { return m[row * PP_LANES + lane]; }
  __device__ __forceinline__ SV sv_at(int row) const {
    return sv(v3(at(row), at(row + 1), at(row + 2)), v3(at(row + 3), at(row + 4), at(row + 5)));
  }
  __device__ __forceinline__ void sv_put(int row, SV x) const {
    at(row) = x.a.x; at(row + 1) = x.a.y; at(row + 2) = x.a.z;
    at(row + 3) = x.b.x; at(row + 4) = x.b.y; at(row + 5) = x.b.z;
  }
};

// Bias acceleration c_j from its stored components (see the row layout).
__device__ __forceinline__ SV c_at(const Lds &L, int j) {
  const V3f z = v3(0.0f, 0.0f, 0.0f);
  if (j < 2) return sv(z, z);
  if (j == 2) return sv(z, v3(L.at(R_C), L.at(R_C + 1), L.at(R_C + 2)));
  if (j <= PALM) return L.sv_at(R_C + 3 + 6 * (j - 3));
  const int r = R_C + 3 + 6 * NARM + 3 * (j - FL);
  return sv(z, v3(L.at(r), L.at(r + 1), L.at(r + 2)));
}
__device__ __forceinline__ void c_put(const Lds &L, int j, SV c) {
  if (j < 2) return;
  if (j == 2) {
    L.at(R_C) = c.b.x; L.at(R_C + 1) = c.b.y; L.at(R_C + 2) = c.b.z;
  } else if (j <= PALM) {
    L.sv_put(R_C + 3 + 6 * (j - 3), c);
  } else {
    const int r = R_C + 3 + 6 * NARM + 3 * (j - FL);
    L.at(r) = c.b.x; L.at(r + 1) = c.b.y; L.at(r + 2) = c.b.z;
  }
}
// The LDS row of component i (0..5 over [w; v]) of c_J, for the components
// c_mask<J>() keeps (the rows c_put writes); the masked-out ones are zero.
template <int J> constexpr int c_row(int i) {
  return J == 2 ? R_C + (i - 3)
                : (J <= PALM ? R_C + 3 + 6 * (J - 3) + i : R_C + 3 + 6 * NARM + 3 * (J - FL) + (i - 3));
}
template <int J> __device__ __forceinline__ void c_put_t(const Lds &L, SV c) {
  constexpr unsigned M = c_mask<J>();
  const float x[6] = {c.a.x, c.a.y, c.a.z, c.b.x, c.b.y, c.b.z};
  sfor<0, 6>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    if constexpr ((M >> i) & 1u) L.at(c_row<J>(i)) = x[i];
  });
}
// The specialised passes leave the rows of c_J's structural zeros unwritten;
// they hold the cosine and sine of revolute joint J (2..PALM) from the first
// pass for the second and third: an arm joint's in its own body's axis rows,
// the base yaw's in body 2's zero row and finger FL's.
template <int J> constexpr int cs_row(int which) {
  return J == 2 ? (which == 0 ? c_row<2>(3 + rmx::kax(2)) : c_row<FL>(3 + rmx::kax(FL)))
                : c_row<J>(which == 0 ? rmx::kax(J) : 3 + rmx::kax(J));
}
// those rows are outside the masks of the components c_put_t writes
static_assert(!((c_mask<2>() >> (3 + rmx::kax(2))) & 1u) && !((c_mask<FL>() >> (3 + rmx::kax(FL))) & 1u),
              "spare rows for the base yaw's cosine and sine");
template <int J> __device__ __forceinline__ void cs_put_t(const Lds &L, const JT &X) {
  static_assert(J >= 2 && J <= PALM && rmx::rev(J), "revolute joints 2..PALM");
  static_assert(J == 2 || (!((c_mask<J>() >> rmx::kax(J)) & 1u) && !((c_mask<J>() >> (3 + rmx::kax(J))) & 1u)),
                "spare rows of an arm body");
  L.at(cs_row<J>(0)) = X.c;
  L.at(cs_row<J>(1)) = X.s;
}
template <int J> __device__ __forceinline__ SV c_get_t(const Lds &L) {
  constexpr unsigned M = c_mask<J>();
  float x[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  sfor<0, 6>([&](auto ic) {
    constexpr int i = decltype(ic)::value;
    if constexpr ((M >> i) & 1u) x[i] = L.at(c_row<J>(i));
  });
  return sv(v3(x[0], x[1], x[2]), v3(x[3], x[4], x[5]));
}

// Sum over the G (1, 2, 4, 8 or 16) adjacent lanes that share an environment,
// by a butterfly: quad permutations for lane distances 1 and 2, swizzles (xor
// within 32 lanes) for 4 and 8.  Each level adds the same two operands on both
// lanes of a pair, so every lane of the group ends with the same bits and the
// group's lanes keep identical state.  The group's lanes are all active or
// all inactive.
__device__ __forceinline__ float group_sum(float v, int G) {
  if (G >= 2) v = v + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true));
  if (G >= 4) v = v + __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, true));
  if (G >= 8) v = v + __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x101F));
  if (G >= 16) v = v + __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x201F));
  return v;
}
__device__ __forceinline__ V3f group_sum(V3f v, int G) {
  return v3(group_sum(v.x, G), group_sum(v.y, G), group_sum(v.z, G));
}

// With G = 8 or 16 lanes, a contact test split across G / 4 lanes: the
// corners lane gi takes (G 8: even or odd indices; G 16: indices congruent to
// gi / 4 mod 4).
__device__ __forceinline__ unsigned corner_part(int gi, int G) {
  return G == 8 ? 0x55u << ((gi >> 2) & 1) : G == 16 ? 0x11u << ((gi >> 2) & 3) : 0xFFu;
}

// Joint reference row (both fingers share one).
__device__ __forceinline__ int qref_row(int j) { return R_QREF + (j < FL ? j : FL); }

// Outcome of one rollout: Problem 2's cost and tier, the object's final pose
// (p, q) and the control steps simulated (T, or fewer after an early stop or
// a divergence).
struct EnvOut {
  float cost;
  int tier, steps;
  float pose[7];
};

// Rolls out parameter rows of Z (16 parameters for pick-and-place, 12 for
// move-push), one after another on this lane: first row0 (if live0), then
// each row that `claim` hands out when a rollout ends, until it hands out
// none.  Each rollout runs with the object's friction `mu_obj` (0: the
// per-class coefficients) and mass `om`, and (TRACE) writes its per-step
// trace; its outcome goes to finish(EnvOut, row).  Returns the control steps
// this lane simulated.  The wave steps its lanes together, one control step
// per loop iteration, each lane at its own step of its own rollout, so a lane
// whose rollout ends can start the next while the others run on.
//   claim(need, row, live): called by every lane of the wave at the same
//     point; for each lane with `need` set it stores the next row in `row`
//     and sets `live`, or clears `live` when there is none.
// `lds_mem` is the block's R_ROWS x PP_LANES float array and `lane` this
// lane's column in it.  The scene and its derived constants come from `st`.
// G adjacent lanes (1, 2, 4, 8 or 16; gi this lane's place among them) run
// the same environment: each keeps the whole state, takes every G-th contact
// test of the object and the base against the world, and a share of the
// finger-object tests (G 2: one finger; G 4: one finger, one direction; G 8,
// 16: that, on part of the corners);
// the forces are then summed over the group, whose lanes therefore start and
// end their rollouts together.  With G = 1 the sums run in the original
// order; the MULTI = false instance compiles G = 1 in.
template <bool TRACE, bool MULTI, bool SPEC, class Claim, class Finish>
__device__ __forceinline__ int robot_env(CDevState *st, const float *__restrict__ Z, long row0, bool live0,
                                          float mu_obj, float om, float *lds_mem, int lane, int gi_in, int G_in,
                                          float *__restrict__ trace, int trace_steps, Claim claim, Finish finish) {
  // !MULTI: one lane per environment, known at compile time
  const int G = MULTI ? G_in : 1, gi = MULTI ? gi_in : 0;
  CScene &sc = st->scene;
  CConsts &sk = st->sk;
  const Lds L{lds_mem, lane};
  const bool pnp = sc.kind == CEM_SCENE_PICKPLACE;
  const int n_act = pnp ? 4 : 2, n_par = pnp ? 16 : 12;
  const bool mu_drawn = mu_obj > 0.0f;
  const float mu_o_ground = mu_drawn ? mu_obj : sc.mu_ground, mu_o_tool = mu_drawn ? mu_obj : sc.mu_tool;
  const float h = sc.dt / (float)sc.substeps;
  const float dt = sc.dt;
  const float g = sc.gravity;
  const float kc = sc.k_contact, damp = sc.c_contact, eps2 = sc.eps_v * sc.eps_v;
  const float wc = sc.omega_c, zeta = sc.zeta;
  const V3f ohe = v3(sc.obj_half[0], sc.obj_half[1], sc.obj_half[2]);
  const float inv_om = 1.0f / om;
  const V3f oIb = v3(om * (ohe.y * ohe.y + ohe.z * ohe.z) / 3.0f, om * (ohe.x * ohe.x + ohe.z * ohe.z) / 3.0f,
                     om * (ohe.x * ohe.x + ohe.y * ohe.y) / 3.0f);
  const V3f inv_oIb = v3(1.0f / oIb.x, 1.0f / oIb.y, 1.0f / oIb.z);
  const V3f gv = v3(0.0f, 0.0f, -g);

  Params4 zp;
  FreeBody ob;

  // controller state
  int act = 0, t_start = 0;
  unsigned ok_bits = 0;
  float qstart[NARM + 3], qa[NARM], qb[NARM];
  V3f ptarget = v3(0.0f, 0.0f, 0.0f);
  float base_from[3] = {0.0f, 0.0f, 0.0f}, base_to[3] = {0.0f, 0.0f, 0.0f}, t_move = 1.0f;
  float Ta = sc.t_approach, Td = sc.t_descend, Tl = sc.t_lift, Tp = sc.t_transfer, Tq = dt;
  float push_nominal = 0.0f;
  bool push_ready = false;
  float finger_cmd = sc.finger_open;
  bool touchL = false, touchR = false;
  int unsuccessful = 0;
#pragma unroll
  for (int j = 0; j < NARM; ++j) { qa[j] = 0.0f; qb[j] = 0.0f; }

  auto load_q = [&](float (&qc)[NJ]) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) qc[j] = L.at(R_Q + j);
  };
  auto span = [&](const float (&from)[NARM], const float (&to)[NARM], float nominal) {
    float m = 0.0f;
#pragma unroll
    for (int j = 0; j < NARM; ++j) m = fmaxf(m, fabsf(to[j] - from[j]));
    return fmaxf(nominal, m / sc.joint_speed_max);
  };

  auto start_action = [&](int a, int t) {
    float q[NJ];
    load_q(q);
    t_start = t;
#pragma unroll
    for (int j = 0; j < NARM + 3; ++j) qstart[j] = q[j];
    float pz[4];
    action_params(zp, a, pz);
    const int kind = act_kind(pnp, a);
    if (kind == MOVE) {
      base_from[0] = q[0]; base_from[1] = q[1]; base_from[2] = q[2];
      const float dpsi = wrap_pi(pz[2] - q[2]);
      base_to[0] = pz[0]; base_to[1] = pz[1]; base_to[2] = q[2] + dpsi;
      const float v = fmaxf(sc.base_vmin, fminf(sc.base_vmax, pz[3]));
      const float dx = pz[0] - q[0], dy = pz[1] - q[1];
      const float Lm = sqrtf(dx * dx + dy * dy);
      t_move = fmaxf(fmaxf(Lm / v, fabsf(dpsi) / sc.base_wmax), dt);
    } else if (kind == PUSH) {
      // parameters: block 1 = start point xyz, heading; block 2 = distance, speed, approach height, gripper yaw
      float pw[4];
      action_params(zp, 2, pw);
      float sg, cg, sh, ch;
      sincosf(pw[3], &sg, &cg);
      sincosf(pz[3], &sh, &ch);
      M3f Rt;
      Rt.r0 = v3(cg, sg, 0.0f);
      Rt.r1 = v3(sg, -cg, 0.0f);
      Rt.r2 = v3(0.0f, 0.0f, -1.0f);
      const V3f ps = v3(pz[0], pz[1], pz[2]);
      const float dist = fmaxf(0.0f, fminf(sc.push_dmax, pw[0]));
      const float vp = fmaxf(sc.push_vmin, fminf(sc.push_vmax, pw[1]));
      const float dz = fmaxf(0.0f, pw[2]);
      const V3f pe = ps + dist * v3(ch, sh, 0.0f);
      float qs[NARM];
#pragma unroll
      for (int j = 0; j < NARM; ++j) qs[j] = q[ARM0 + j];
      ik_dls<SPEC>(sc, q, ps + v3(0.0f, 0.0f, dz), Rt);
#pragma unroll
      for (int j = 0; j < NARM; ++j) qa[j] = q[ARM0 + j];
      ik_dls<SPEC>(sc, q, ps, Rt);
#pragma unroll
      for (int j = 0; j < NARM; ++j) qb[j] = q[ARM0 + j];
      // the end-of-line anchor (IK from (base at action start, qb) toward pe)
      // is solved when the push phase begins, into qa, which that phase no
      // longer needs
      Ta = span(qs, qa, sc.t_approach);
      Td = span(qa, qb, sc.t_descend);
      push_nominal = dist / vp;
      push_ready = false;
      ptarget = pe;
    } else {
      M3f Rt;
      V3f pfin, pgoal;
      if (kind == PICK) {
        // grasp orientation from the normalised quaternion parameter
        float w = pz[0], x = pz[1], y = pz[2], z = pz[3];
        const float n2 = w * w + x * x + y * y + z * z;
        if (!(n2 > 1e-12f)) { w = 1.0f; x = 0.0f; y = 0.0f; z = 0.0f; }
        else {
          const float inv = 1.0f / sqrtf(n2);
          w *= inv; x *= inv; y *= inv; z *= inv;
        }
        Rt = rot_of(Q4f{w, x, y, z});
        pgoal = ob.p;
        pfin = pgoal - sc.pregrasp * v3(Rt.r0.z, Rt.r1.z, Rt.r2.z);
      } else {
        float sy, cy;
        sincosf(pz[3], &sy, &cy);
        Rt.r0 = v3(cy, sy, 0.0f);
        Rt.r1 = v3(sy, -cy, 0.0f);
        Rt.r2 = v3(0.0f, 0.0f, -1.0f);
        pfin = v3(pz[0], pz[1], pz[2]);
        pgoal = pfin;
      }
      float qs[NARM];
#pragma unroll
      for (int j = 0; j < NARM; ++j) qs[j] = q[ARM0 + j];
      ik_dls<SPEC>(sc, q, pfin, Rt);
#pragma unroll
      for (int j = 0; j < NARM; ++j) qa[j] = q[ARM0 + j];
      if (kind == PICK) {
        ik_dls<SPEC>(sc, q, pgoal, Rt);
#pragma unroll
        for (int j = 0; j < NARM; ++j) qb[j] = q[ARM0 + j];
        Ta = span(qs, qa, sc.t_approach);
        Td = span(qa, qb, sc.t_descend);
        Tl = span(qb, qa, sc.t_lift);
      } else {
        Tp = span(qs, qa, sc.t_transfer);
      }
      ptarget = pfin;
    }
  };


  // a rollout from its first step: row r's parameters, the robot at q0 and at
  // rest, the object at its start pose, the controllers and the success record
  // cleared, the first action started
  auto init_plan = [&](long r) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int i = 0; i < 4; ++i) zp.v[a][i] = 4 * a + i < n_par ? Z[r * n_par + 4 * a + i] : 0.0f;
    for (int j = 0; j < NJ; ++j) {
      L.at(R_Q + j) = sc.q0[j];
      L.at(R_QD + j) = 0.0f;
      if (j <= FL) L.at(R_QREF + j) = sc.q0[j];
    }
    ob.p = v3(sc.obj_pos0[0], sc.obj_pos0[1], sc.obj_pos0[2] - om * g / (4.0f * kc));
    {
      float s, c;
      sincosf(0.5f * sc.obj_yaw0, &s, &c);
      ob.q = Q4f{c, 0.0f, 0.0f, s};
    }
    ob.v = v3(0.0f, 0.0f, 0.0f);
    ob.w = v3(0.0f, 0.0f, 0.0f);
    act = 0;
    t_start = 0;
    ok_bits = 0;
    ptarget = v3(0.0f, 0.0f, 0.0f);
#pragma unroll
    for (int c = 0; c < 3; ++c) { base_from[c] = 0.0f; base_to[c] = 0.0f; }
    t_move = 1.0f;
    Ta = sc.t_approach; Td = sc.t_descend; Tl = sc.t_lift; Tp = sc.t_transfer; Tq = dt;
    push_nominal = 0.0f;
    push_ready = false;
    finger_cmd = sc.finger_open;
    touchL = false;
    touchR = false;
    unsuccessful = 0;
#pragma unroll
    for (int j = 0; j < NARM; ++j) { qa[j] = 0.0f; qb[j] = 0.0f; }
    start_action(0, 0);
  };

  long row = row0;
  bool live = live0;
  bool diverged = false;
  int steps = sc.horizon, calm = 0, t = 0, total = 0;
  if (live) init_plan(row);
  while (__ballot(live) != 0ull) {
    bool ended = false;
    if (live) {
      // ---- action sequencing (control rate) ----
      if (act < n_act) {
        float q[NJ];
        load_q(q);
        const float tau = (float)(t - t_start) * dt;
        const int kind = act_kind(pnp, act);
        bool succ;
        if (kind == MOVE) {
          float pz[4];
          action_params(zp, act, pz);
          const float dx = q[0] - pz[0], dy = q[1] - pz[1];
          succ = sqrtf(dx * dx + dy * dy) <= sc.base_tol && fabsf(wrap_pi(q[2] - pz[2])) <= sc.yaw_tol;
        } else {
          M3f Rw[PALM + 1];
          V3f pw[PALM + 1];
          if constexpr (SPEC) chain_fk_t(q, Rw, pw);
          else chain_fk(sc, q, Rw, pw);
          const V3f pe = ee_point(sc, Rw[PALM], pw[PALM]);
          const V3f de = pe - ptarget;
          const bool near = sqrtf(dot(de, de)) <= sc.ee_tol;
          if (kind == PICK) {
            const float tend = Ta + Td + sc.t_close + Tl;
            const V3f op = mulT(Rw[PALM], ob.p - pw[PALM]);
            const bool between = op.y < q[FL] && op.y > -q[FR];
            succ = tau >= tend && touchL && touchR && between && near;
          } else if (kind == PUSH) {
            succ = tau >= Ta + Td + Tq + sc.t_release && near;
          } else {
            succ = tau >= Tp + sc.t_release && near;
          }
        }
        const float tout = kind == MOVE   ? sc.timeout_move
                           : kind == PICK ? sc.timeout_pick
                           : kind == PUSH ? sc.timeout_push
                                          : sc.timeout_place;
        if (succ || tau >= tout) {
          if (succ) ok_bits |= 1u << act;
          ++act;
          if (!succ && sc.fail_stop) {
            // the plan can no longer become feasible: it ends before step t
            ended = true;
            steps = t;
          } else if (act < n_act) {
            start_action(act, t);
          }
        }
      }
      if (!ended) {
        if (act < n_act) ++unsuccessful;
        // ---- references ----
        if (act < n_act) {
          const float tau = (float)(t - t_start) * dt;
          const int kind = act_kind(pnp, act);
          float r[NARM + 3];
          if (kind == MOVE) {
            const float sft = smooth01(tau / t_move);
#pragma unroll
            for (int c = 0; c < 3; ++c) r[c] = base_from[c] + sft * (base_to[c] - base_from[c]);
#pragma unroll
            for (int j = 0; j < NARM; ++j) r[3 + j] = qstart[ARM0 + j];
          } else if (kind == PICK) {
            const float Tc = sc.t_close;
#pragma unroll
            for (int c = 0; c < 3; ++c) r[c] = qstart[c];
#pragma unroll
            for (int j = 0; j < NARM; ++j) {
              float v;
              const float s0 = qstart[ARM0 + j];
              if (tau < Ta) v = s0 + smooth01(tau / Ta) * (qa[j] - s0);
              else if (tau < Ta + Td) v = qa[j] + smooth01((tau - Ta) / Td) * (qb[j] - qa[j]);
              else if (tau < Ta + Td + Tc) v = qb[j];
              else if (tau < Ta + Td + Tc + Tl) v = qb[j] + smooth01((tau - Ta - Td - Tc) / Tl) * (qa[j] - qb[j]);
              else v = qa[j];
              r[3 + j] = v;
            }
            finger_cmd = tau < Ta + Td ? sc.finger_open : sc.finger_closed;
          } else if (kind == PUSH) {
            if (tau >= Ta + Td && !push_ready) {
              float pw[4];
              action_params(zp, 2, pw);
              float sg, cg;
              sincosf(pw[3], &sg, &cg);
              M3f Rt;
              Rt.r0 = v3(cg, sg, 0.0f);
              Rt.r1 = v3(sg, -cg, 0.0f);
              Rt.r2 = v3(0.0f, 0.0f, -1.0f);
              float qq[NJ];
#pragma unroll
              for (int c = 0; c < 3; ++c) qq[c] = qstart[c];
#pragma unroll
              for (int j = 0; j < NARM; ++j) qq[ARM0 + j] = qb[j];
              qq[FL] = 0.0f;
              qq[FR] = 0.0f;
              ik_dls<SPEC>(sc, qq, ptarget, Rt);
#pragma unroll
              for (int j = 0; j < NARM; ++j) qa[j] = qq[ARM0 + j];
              Tq = fmaxf(span(qb, qa, push_nominal), dt);
              push_ready = true;
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) r[c] = qstart[c];
#pragma unroll
            for (int j = 0; j < NARM; ++j) {
              // qa: the pre-push pose until the push phase, then the end-of-line anchor
              float v;
              const float s0 = qstart[ARM0 + j];
              if (tau < Ta) v = s0 + smooth01(tau / Ta) * (qa[j] - s0);
              else if (tau < Ta + Td) v = qa[j] + smooth01((tau - Ta) / Td) * (qb[j] - qa[j]);
              else if (tau < Ta + Td + Tq) v = qb[j] + smooth01((tau - Ta - Td) / Tq) * (qa[j] - qb[j]);
              else v = qa[j];
              r[3 + j] = v;
            }
            finger_cmd = tau < Ta + Td + Tq ? sc.finger_closed : sc.finger_open;
          } else {
#pragma unroll
            for (int c = 0; c < 3; ++c) r[c] = qstart[c];
#pragma unroll
            for (int j = 0; j < NARM; ++j) {
              const float s0 = qstart[ARM0 + j];
              r[3 + j] = tau < Tp ? s0 + smooth01(tau / Tp) * (qa[j] - s0) : qa[j];
            }
            finger_cmd = tau < Tp ? sc.finger_closed : sc.finger_open;
          }
#pragma unroll
          for (int j = 0; j < NARM + 3; ++j) L.at(R_QREF + j) = r[j];
        }
        L.at(R_QREF + FL) = finger_cmd;
      }
    }
    if (live && !ended) {
    for (int si = 0; si < sc.substeps; ++si) {
      const bool last = si == sc.substeps - 1;
      // ---- the object against the world (ground, static boxes) ----
      Box OB;
      OB.p = ob.p;
      OB.R = rot_of(ob.q);
      OB.h = ohe;
      Wrench W{v3(0.0f, 0.0f, 0.0f), v3(0.0f, 0.0f, 0.0f)};
      // test u: 0 the ground, 1 + b static box b; this lane takes every G-th,
      // or, with 8 or 16 lanes and at most four tests, every 4th on the part
      // of the corners that gi / 4 picks
      const bool w_halves = G >= 8 && sc.n_static + 1 <= 4;
      const int w_step = w_halves ? 4 : G;
      const unsigned w_mask = w_halves ? corner_part(gi, G) : 0xFFu;
      // Contacts are formed in the frame of the box whose face they press on
      // (there the normal is an axis): the object's velocity in its own frame,
      // and the force and moment sums of the contacts on the object's faces in
      // that frame (FO, TO, about its centre), rotated into the world once
      // after the fingers' contacts
      const V3f vO = mulT(OB.R, ob.v), wO = mulT(OB.R, ob.w);
      V3f FO = v3(0.0f, 0.0f, 0.0f), TO = v3(0.0f, 0.0f, 0.0f);
      const int u0 = gi & (w_step - 1);
      if (u0 == 0) box_ground(ob, OB.R, ohe, kc, damp, mu_o_ground, eps2, W, w_mask);
      // The static boxes this lane takes that no face axis separates from the
      // object, then one pass per such box of a lane in ascending order: lanes
      // whose near boxes differ share passes (a wave runs as many as its lane
      // with the most near boxes, not one per box that any lane is near).
      unsigned near = 0u;
      for (int u = u0 == 0 ? w_step : u0; u <= sc.n_static; u += w_step) {
        const Box SB = static_box(sc, sk, u - 1);
        bool sep;
        if (sk.st_axis[u - 1]) sep = face_separated(rel_of_axis(OB, SB), ohe, SB.h);  // an unrotated box
        else sep = face_separated(rel_of(OB, SB), ohe, SB.h);
        if (!sep) near |= 1u << (u - 1);
      }
      while (near != 0u) {  // at most CEM_MAX_STATIC passes
        const int b = __builtin_ctz(near);
        near &= near - 1u;
        const Box SB = static_box(sc, sk, b);
        const float mu = mu_drawn ? mu_obj : (sc.st_ramp[b] ? sc.mu_ramp : sc.mu_static);
        const Rel r = rel_of(OB, SB);
        // object vertices in the static box (A = object), in the box's frame,
        // where the object's centre is r.t
        const V3f vB = mulT(SB.R, ob.v), wB = mulT(SB.R, ob.w);
        V3f F = v3(0.0f, 0.0f, 0.0f), T = v3(0.0f, 0.0f, 0.0f);
        verts_in_box_b(r, ohe, SB.h, [&](V3f xb, int ax, float sg, float d) {
          const V3f ro = xb - r.t;
          const V3f f = contact_force_b(ax, sg, d, vB + cross(wB, ro), kc, damp, mu, eps2);
          F = F + f;
          T = T + cross(ro, f);
        }, w_mask);
        W.f = W.f + mul(SB.R, F);
        W.t = W.t + mul(SB.R, T);
        // static-box vertices in the object (A = static box, the object
        // receives the negative), where one can reach into it
        if (corners_reach(r, ohe, SB.h))
          verts_in_box_b(rel_swap(r), SB.h, ohe, [&](V3f xb, int ax, float sg, float d) {
            const V3f f = -contact_force_b(ax, sg, d, v3(0.0f, 0.0f, 0.0f) - (vO + cross(wO, xb)), kc, damp, mu, eps2);
            FO = FO + f;
            TO = TO + cross(xb, f);
          }, w_mask);
      }

      // ---- ABA pass 1 (root to leaves): poses, velocities, bias terms ----
      // The chain (bodies 0..PALM), then the fingers, children of the palm:
      // separate loops, so the parent's pose needs no per-body select.
      M3f Rw;  // world pose and velocity of the latest chain body (the palm's after the chain)
      V3f pw = v3(0.0f, 0.0f, 0.0f);
      SV vprev = sv(v3(0.0f, 0.0f, 0.0f), v3(0.0f, 0.0f, 0.0f));
      Rw.r0 = v3(1.0f, 0.0f, 0.0f); Rw.r1 = v3(0.0f, 1.0f, 0.0f); Rw.r2 = v3(0.0f, 0.0f, 1.0f);
      M3f Rw2;  // the base link's pose and velocity, for its contacts
      V3f pw2;
      SV v2;
      M3f Rf[2];  // SPEC: the fingers' poses and velocities from the first pass
      V3f pf[2];
      SV vf[2];
      if constexpr (SPEC) {
        // the model's bodies in order, unrolled; the chain's pose and velocity
        // stay the palm's once the fingers come
        sfor<0, NJ>([&](auto jc) {
          constexpr int J = decltype(jc)::value;
          const float qj = L.at(R_Q + J), qdj = L.at(R_QD + J);
          const JT X = joint_t<J>(qj);
          if constexpr (J >= 2 && J <= PALM) cs_put_t<J>(L, X);
          const M3f Rb = rot_right_k<rmx::kax(J)>(Rw, X.c, X.s);
          V3f pb;
          if constexpr (rmx::rev(J)) pb = pw + rot_org<J>(Rw);
          else pb = pw + mul(Rw, X.r);
          const SV vJ = s_vec_t<J>(qdj);
          SV vb;
          if constexpr (J == 0) vb = vJ;
          else vb = x_motion_t<J>(X, vprev) + vJ;
          c_put_t<J>(L, crm_s<J>(vb, qdj));
          L.sv_put(R_P + 6 * J, crf(vb, body_mul<J>(vb)));
          if constexpr (J <= PALM) {
            Rw = Rb;
            pw = pb;
            vprev = vb;
          }
          if constexpr (J == BASEB) {
            Rw2 = Rb;
            pw2 = pb;
            v2 = vb;
          }
          if constexpr (J >= FL) {
            Rf[J - FL] = Rb;
            pf[J - FL] = pb;
            vf[J - FL] = vb;
          }
        });
      } else {
        auto pass1 = [&](int j, const M3f &Rp, V3f pp, const SV &vp, M3f &Rb, V3f &pb, SV &vb) {
          const float qj = L.at(R_Q + j);
          const JT X = joint_of(sc, j, qj);
          Rb = rot_right(Rp, X);
          pb = pp + mul(Rp, X.r);
          const SV vJ = s_vec(sc, j, L.at(R_QD + j));
          vb = (j == 0 ? sv(v3(0.0f, 0.0f, 0.0f), v3(0.0f, 0.0f, 0.0f)) : x_motion(X, vp)) + vJ;
          c_put(L, j, crm(vb, vJ));
          L.sv_put(R_P + 6 * j, crf(vb, sym_mul(inertia_of(sk, j), vb)));
        };
        for (int j = 0; j <= BASEB; ++j) {
          M3f Rb;
          V3f pb;
          SV vb;
          pass1(j, Rw, pw, vprev, Rb, pb, vb);
          Rw = Rb;
          pw = pb;
          vprev = vb;
        }
        Rw2 = Rw;  // the base link's pose and velocity, for its contacts
        pw2 = pw;
        v2 = vprev;
        for (int j = BASEB + 1; j <= PALM; ++j) {
          M3f Rb;
          V3f pb;
          SV vb;
          pass1(j, Rw, pw, vprev, Rb, pb, vb);
          Rw = Rb;
          pw = pb;
          vprev = vb;
        }
        for (int j = FL; j <= FR; ++j) {
          M3f Rb;
          V3f pb;
          SV vb;
          pass1(j, Rw, pw, vprev, Rb, pb, vb);
        }
      }

      // ---- contacts on the base link and the fingers: world forces become body
      // spatial forces, taken off those bodies' bias forces ----
      {
        auto link_box = [&](int j, const M3f &Rb, V3f pb) {
          Box LB;
          LB.p = pb + mul(Rb, v3(sc.b_com[j][0], sc.b_com[j][1], sc.b_com[j][2]));
          LB.R = Rb;
          LB.h = v3(sc.b_half[j][0], sc.b_half[j][1], sc.b_half[j][2]);
          return LB;
        };
        // the base link against the static boxes
        {
          Box LB;
          V3f com;
          if constexpr (SPEC) {  // the model's link box, its centre's offset with the structural zeros left out
            com = v3(rm::COM[BASEB][0], rm::COM[BASEB][1], rm::COM[BASEB][2]);
            LB.p = pw2 + rot_com<BASEB>(Rw2);
            LB.R = Rw2;
            LB.h = v3(rm::HALF[BASEB][0], rm::HALF[BASEB][1], rm::HALF[BASEB][2]);
          } else {
            LB = link_box(BASEB, Rw2, pw2);
            com = v3(sc.b_com[BASEB][0], sc.b_com[BASEB][1], sc.b_com[BASEB][2]);
          }
          // the spatial force on the link in its body frame (moment about the
          // body origin); the link box's frame is the body's, offset by com
          V3f fm = v3(0.0f, 0.0f, 0.0f), ff = v3(0.0f, 0.0f, 0.0f);
          // every G-th static box, or with 8 or 16 lanes and at most four
          // boxes every 4th on part of the corners, as for the object above
          const bool b_halves = G >= 8 && sc.n_static <= 4;
          const int b_step = b_halves ? 4 : G;
          const unsigned b_mask = b_halves ? corner_part(gi, G) : 0xFFu;
          // the near boxes first, then one pass per near box of a lane, as
          // for the object above
          unsigned near = 0u;
          for (int b = gi & (b_step - 1); b < sc.n_static; b += b_step) {
            const Box SB = static_box(sc, sk, b);
            bool sep;
            if (sk.st_axis[b]) sep = face_separated(rel_of_axis(LB, SB), LB.h, SB.h);  // an unrotated box
            else sep = face_separated(rel_of(LB, SB), LB.h, SB.h);
            if (!sep) near |= 1u << b;
          }
          while (near != 0u) {  // at most CEM_MAX_STATIC passes
            const int b = __builtin_ctz(near);
            near &= near - 1u;
            const Box SB = static_box(sc, sk, b);
            const Rel r = rel_of(LB, SB);
            // link vertices in the static box, in the box's frame: the body
            // origin at q, the link's velocity (M v2) there
            const V3f q = r.t - mul(r.M, com), wa = mul(r.M, v2.a), wb = mul(r.M, v2.b);
            V3f F = v3(0.0f, 0.0f, 0.0f), T = v3(0.0f, 0.0f, 0.0f);
            verts_in_box_b(r, LB.h, SB.h, [&](V3f xb, int ax, float sg, float d) {
              const V3f ro = xb - q;
              const V3f f = contact_force_b(ax, sg, d, wb + cross(wa, ro), kc, damp, sc.mu_static, eps2);
              F = F + f;
              T = T + cross(ro, f);
            }, b_mask);
            ff = ff + mulT(r.M, F);
            fm = fm + mulT(r.M, T);
            // static-box vertices in the link, in the body frame, where one
            // can reach into it
            if (corners_reach(r, LB.h, SB.h))
              verts_in_box_b(rel_swap(r), SB.h, LB.h, [&](V3f xb, int ax, float sg, float d) {
                const V3f ro = xb + com;
                const V3f f = -contact_force_b(ax, sg, d, v3(0.0f, 0.0f, 0.0f) - (v2.b + cross(v2.a, ro)), kc, damp,
                                               sc.mu_static, eps2);
                ff = ff + f;
                fm = fm + cross(ro, f);
              }, b_mask);
          }
          if (G > 1) {
            fm = group_sum(fm, G);
            ff = group_sum(ff, G);
          }
          L.sv_put(R_P + 6 * BASEB, L.sv_at(R_P + 6 * BASEB) - sv(fm, ff));
        }
        // the fingers against the object (their pose again from the palm's);
        // G 1 takes both fingers, G 2 finger FL + gi, G 4 finger FL + gi / 2
        // in one direction (bit 0 of dirs: finger vertices in the object,
        // bit 1: object vertices in the finger), G 8 and 16 the same on part
        // of the corners
        const int jf0 = G == 1 ? FL : FL + (G == 2 ? gi : (gi >> 1) & 1), jf1 = G == 1 ? FR : jf0;
        const int dirs = G <= 2 ? 3 : 1 << (gi & 1);
        const unsigned f_mask = corner_part(gi, G);  // 8 or 16 lanes: part of the corners each
        SV part = sv(v3(0.0f, 0.0f, 0.0f), v3(0.0f, 0.0f, 0.0f));  // G > 1: this lane's body-frame share
        bool part_any = false;
        for (int j = jf0; j <= jf1; ++j) {
          M3f Rb;
          V3f pb;
          SV vb;
          if constexpr (SPEC) {
            Rb = j == FL ? Rf[0] : Rf[1];
            pb = j == FL ? pf[0] : pf[1];
            vb = j == FL ? vf[0] : vf[1];
          } else {
            const JT X = joint_of(sc, j, L.at(R_Q + j));
            Rb = rot_right(Rw, X);
            pb = pw + mul(Rw, X.r);
            vb = x_motion(X, vprev) + s_vec(sc, j, L.at(R_QD + j));
          }
          Box LB;
          V3f com;
          if constexpr (SPEC) {  // the model's finger boxes: centres of mass off the x axis
            static_assert(rm::COM[FL][0] == 0.0f && rm::COM[FR][0] == 0.0f, "finger centres of mass on x = 0");
            const bool left = j == FL;
            com = left ? v3(rm::COM[FL][0], rm::COM[FL][1], rm::COM[FL][2]) : v3(rm::COM[FR][0], rm::COM[FR][1], rm::COM[FR][2]);
            LB.p = pb + (com.y * col(Rb, 1) + com.z * col(Rb, 2));
            LB.R = Rb;
            LB.h = left ? v3(rm::HALF[FL][0], rm::HALF[FL][1], rm::HALF[FL][2])
                        : v3(rm::HALF[FR][0], rm::HALF[FR][1], rm::HALF[FR][2]);
          } else {
            LB = link_box(j, Rb, pb);
            com = v3(sc.b_com[j][0], sc.b_com[j][1], sc.b_com[j][2]);
          }
          // the spatial force on the finger in its body frame (the finger
          // box's frame, offset by com)
          V3f fm = v3(0.0f, 0.0f, 0.0f), ff = v3(0.0f, 0.0f, 0.0f);
          const Rel r = rel_of(LB, OB);
          bool any = false;
          if (!face_separated(r, LB.h, ohe)) {
            // finger vertices in the object (A = finger, B = object), in the
            // object's frame: the finger's origin at q, its velocity (M vb) there
            if (dirs & 1) {
              const V3f q = r.t - mul(r.M, com), wa = mul(r.M, vb.a), wb = mul(r.M, vb.b);
              V3f F = v3(0.0f, 0.0f, 0.0f), T = v3(0.0f, 0.0f, 0.0f);
              verts_in_box_b(r, LB.h, ohe, [&](V3f xb, int ax, float sg, float d) {
                const V3f f = contact_force_b(ax, sg, d, (wb + cross(wa, xb - q)) - (vO + cross(wO, xb)), kc, damp,
                                              mu_o_tool, eps2);
                F = F + f;
                T = T + cross(xb - q, f);
                FO = FO - f;
                TO = TO - cross(xb, f);
                any = true;
              }, f_mask);
              ff = ff + mulT(r.M, F);
              fm = fm + mulT(r.M, T);
            }
            // object vertices in the finger (A = object, B = finger), in the
            // finger's frame: the object's centre at rs.t, its velocity there;
            // only where a corner of the object can reach into the finger
            if ((dirs & 2) && corners_reach(r, LB.h, ohe)) {
              const Rel rs = rel_swap(r);
              const V3f vF = mulT(r.M, vO), wF = mulT(r.M, wO);
              V3f F = v3(0.0f, 0.0f, 0.0f), T = v3(0.0f, 0.0f, 0.0f);
              verts_in_box_b(rs, ohe, LB.h, [&](V3f xb, int ax, float sg, float d) {
                const V3f ro = xb + com;
                const V3f f = contact_force_b(ax, sg, d, (vF + cross(wF, xb - rs.t)) - (vb.b + cross(vb.a, ro)), kc,
                                              damp, mu_o_tool, eps2);
                F = F + f;
                T = T + cross(xb - rs.t, f);
                ff = ff - f;
                fm = fm - cross(ro, f);
                any = true;
              }, f_mask);
              FO = FO + mul(r.M, F);
              TO = TO + mul(r.M, T);
            }
          }
          if (G == 1) {
            if (last) {
              if (j == FL) touchL = any;
              else touchR = any;
            }
            L.sv_put(R_P + 6 * j, L.sv_at(R_P + 6 * j) - sv(fm, ff));
          } else {
            part = sv(fm, ff);
            part_any = any;
          }
        }
        // the object's contacts on its own faces, into the world
        W.f = W.f + mul(OB.R, FO);
        W.t = W.t + mul(OB.R, TO);
        if (G > 1) {
          // each finger's force from the lanes that tested it (the others add
          // exact zeros), the object's wrench from the whole group
          const V3f z = v3(0.0f, 0.0f, 0.0f);
          const bool left = jf0 == FL;
          const SV pL = sv(group_sum(left ? part.a : z, G), group_sum(left ? part.b : z, G));
          const SV pR = sv(group_sum(left ? z : part.a, G), group_sum(left ? z : part.b, G));
          const float aL = group_sum(left && part_any ? 1.0f : 0.0f, G);
          const float aR = group_sum(!left && part_any ? 1.0f : 0.0f, G);
          if (last) {
            touchL = aL > 0.0f;
            touchR = aR > 0.0f;
          }
          L.sv_put(R_P + 6 * FL, L.sv_at(R_P + 6 * FL) - pL);
          L.sv_put(R_P + 6 * FR, L.sv_at(R_P + 6 * FR) - pR);
          W.f = group_sum(W.f, G);
          W.t = group_sum(W.t, G);
        }
      }

      // ---- ABA pass 2 (leaves to root): articulated inertias, U, D, u ----
      // Body j's articulated inertia IA arrives from its children; the
      // fingers start from their own inertia, fold into the palm's (IA8), the
      // palm and the chain bodies fold into their parent's (IAc).  Three loops
      // with the source and destination fixed, so no per-body selects.  The
      // parent's bias force receives its child's share in registers (pA8 for
      // the palm, pAc along the chain) instead of a round trip through LDS.
      if constexpr (SPEC) {
        // the same passes over the model's bodies, unrolled
        Sym6 IA8 = body_sym<PALM>();
        Sym6 IAc;
        SV pA8 = L.sv_at(R_P + 6 * PALM), pAc;
        auto pass2 = [&](auto jc, Sym6 &IA, const SV &pA_in) {
          constexpr int J = decltype(jc)::value;
          const SV pAj = pA_in;
          const float qj = L.at(R_Q + J), qdj = L.at(R_QD + J);
          const float lim = sc.j_inom[J] * sc.accel_max;
          const float tq = fmaxf(-lim, fminf(lim, sc.j_inom[J] * (wc * wc * (L.at(qref_row(J)) - qj) - 2.0f * zeta * wc * qdj)));
          const SV Uj = rmx::sgn(J) * sym_col(IA, rmx::sub_idx(J));
          const float di = __builtin_amdgcn_rcpf(s_comp_t<J>(Uj));  // the hardware reciprocal (about 1 ulp)
          const float u = tq - s_comp_t<J>(pAj);
          L.sv_put(R_P + 6 * J, di * Uj);  // pA of body J is consumed: its row now holds U / D
          L.at(R_UD + J) = u * di;
          if constexpr (J > 0) {
            sym_rank1_t(IA, Uj, di);
            SV pa = pAj + (u * di) * Uj;
            if constexpr (J >= 2) pa = pa + sym_mul_masked<c_mask<J>()>(IA, c_get_t<J>(L));
            JT X;
            if constexpr (J >= 2 && J <= PALM) X = joint_cs<J>(qj, L.at(cs_row<J>(0)), L.at(cs_row<J>(1)));
            else X = joint_t<J>(qj);
            const Sym6 Ip = congruence_t<J>(X, IA);
            if constexpr (J >= FL) {
              pA8 = pA8 + x_force_T_t<J>(X, pa);
              sym_add(IA8, Ip);
            } else {
              pAc = L.sv_at(R_P + 6 * (J - 1)) + x_force_T_t<J>(X, pa);
              IAc = body_plus<J - 1>(Ip);
            }
          }
        };
        sfor_down<FL, FR + 1>([&](auto jc) {
          constexpr int J = decltype(jc)::value;
          Sym6 IA = body_sym<J>();
          pass2(jc, IA, L.sv_at(R_P + 6 * J));
        });
        pass2(std::integral_constant<int, PALM>(), IA8, pA8);
        sfor_down<0, PALM>([&](auto jc) { pass2(jc, IAc, pAc); });

        SV a_prev = sv(v3(0.0f, 0.0f, 0.0f), v3(0.0f, 0.0f, g));  // world: -gravity
        SV a_palm;
        sfor<0, NJ>([&](auto jc) {
          constexpr int J = decltype(jc)::value;
          const float qj = L.at(R_Q + J);
          JT X;
          if constexpr (J >= 2 && J <= PALM) X = joint_cs<J>(qj, L.at(cs_row<J>(0)), L.at(cs_row<J>(1)));
          else X = joint_t<J>(qj);
          const SV ap = x_motion_t<J>(X, J >= FL ? a_palm : a_prev) + c_get_t<J>(L);
          const float qdd = L.at(R_UD + J) - dot6(L.sv_at(R_P + 6 * J), ap);
          const float qdn = L.at(R_QD + J) + h * qdd;
          L.at(R_QD + J) = qdn;
          L.at(R_Q + J) = qj + h * qdn;
          if constexpr (J <= PALM) a_prev = ap + s_vec_t<J>(qdd);
          if constexpr (J == PALM) a_palm = a_prev;
        });
      } else {
        Sym6 IA8 = inertia_of(sk, PALM);
        Sym6 IAc = IA8;
        SV pA8 = L.sv_at(R_P + 6 * PALM), pAc;
        auto pass2 = [&](int j, Sym6 &IA, const SV &pA_in, auto into_palm) {
          constexpr bool TO_PALM = decltype(into_palm)::value;
          const SV pAj = pA_in;
          const float qj = L.at(R_Q + j), qdj = L.at(R_QD + j);
          const float lim = sc.j_inom[j] * sc.accel_max;
          const float tq = fmaxf(-lim, fminf(lim, sc.j_inom[j] * (wc * wc * (L.at(qref_row(j)) - qj) - 2.0f * zeta * wc * qdj)));
          const SV Uj = s_sign(sc, j) * sym_col(IA, s_index(sc, j));
          const float di = __builtin_amdgcn_rcpf(s_comp(sc, j, Uj));  // the hardware reciprocal (about 1 ulp)
          const float u = tq - s_comp(sc, j, pAj);
          L.sv_put(R_P + 6 * j, di * Uj);  // pA of body j is consumed: its row now holds U / D
          L.at(R_UD + j) = u * di;
          if (j > 0) {
            sym_rank1(IA, Uj, di);
            SV pa = pAj + (u * di) * Uj;
            if (j >= 2) pa = pa + sym_mul(IA, c_at(L, j));
            const JT X = joint_of(sc, j, qj);
            const int p = parent_of(j);
            // fold body j into its parent, with the transform specialised to the joint's axis
            auto fold = [&](auto axis) {
              constexpr int K = decltype(axis)::value;
              const Sym6 Ip = congruence_k<K>(X, IA);
              if constexpr (TO_PALM) {
                pA8 = pA8 + x_force_T_k<K>(X, pa);
                sym_add(IA8, Ip);
              } else {
                pAc = L.sv_at(R_P + 6 * p) + x_force_T_k<K>(X, pa);
                IAc = inertia_of(sk, p);
                sym_add(IAc, Ip);
              }
            };
            if (X.k == 0) fold(AxisK<0>());
            else if (X.k == 1) fold(AxisK<1>());
            else fold(AxisK<2>());
          }
        };
        for (int j = FR; j >= FL; --j) {
          Sym6 IA = inertia_of(sk, j);
          pass2(j, IA, L.sv_at(R_P + 6 * j), BoolK<true>());
        }
        pass2(PALM, IA8, pA8, BoolK<false>());
        for (int j = PALM - 1; j >= 0; --j) pass2(j, IAc, pAc, BoolK<false>());

        // ---- ABA pass 3 (root to leaves): accelerations and the joint update ----
        auto pass3 = [&](int j, const SV &a_parent) {
          const float qj = L.at(R_Q + j);
          const JT X = joint_of(sc, j, qj);
          const SV ap = x_motion(X, a_parent) + c_at(L, j);
          const float qdd = L.at(R_UD + j) - dot6(L.sv_at(R_P + 6 * j), ap);
          const float qdn = L.at(R_QD + j) + h * qdd;
          L.at(R_QD + j) = qdn;
          L.at(R_Q + j) = qj + h * qdn;
          return ap + s_vec(sc, j, qdd);
        };
        SV a_prev = sv(v3(0.0f, 0.0f, 0.0f), v3(0.0f, 0.0f, g));  // world: -gravity
        for (int j = 0; j <= PALM; ++j) a_prev = pass3(j, a_prev);
        for (int j = FL; j <= FR; ++j) pass3(j, a_prev);          // the fingers, from the palm's acceleration
      }
      integrate(ob, W, inv_om, oIb, inv_oIb, gv, h, OB.R);
    }
    if (TRACE && t < trace_steps && gi == 0) {
      float *o = trace + (row * trace_steps + t) * CEM_TRACE_ROBOT;
      o[0] = ob.p.x; o[1] = ob.p.y; o[2] = ob.p.z;
      o[3] = ob.q.w; o[4] = ob.q.x; o[5] = ob.q.y; o[6] = ob.q.z;
      o[7] = ob.v.x; o[8] = ob.v.y; o[9] = ob.v.z;
      o[10] = ob.w.x; o[11] = ob.w.y; o[12] = ob.w.z;
      for (int j = 0; j < NJ; ++j) { o[13 + j] = L.at(R_Q + j); o[24 + j] = L.at(R_QD + j); }
    }
      if (!isfinite(ob.p.x) || !isfinite(L.at(R_Q + 0))) {
        diverged = true;
        steps = t + 1;
        ended = true;
      } else {
        if (sc.settle_steps > 0) {
          // early stop: the cost is final once the last action has ended; after
          // settle_steps steps of the object at rest psi_g is read at this step
          const bool at_rest = sqrtf(dot(ob.v, ob.v)) < sc.rest_speed;
          calm = (act >= n_act && at_rest) ? calm + 1 : 0;
          if (calm >= sc.settle_steps) {
            steps = t + 1;
            ended = true;
          }
        }
        if (!ended && t + 1 >= sc.horizon) {
          steps = sc.horizon;
          ended = true;
        }
      }
      ++t;
    }
    if (live && ended) {
      // goal psi_g: the object at rest, on the goal table's top face or with its centre inside the goal box
      bool goal = false;
      const bool rest = sqrtf(dot(ob.v, ob.v)) < sc.rest_speed;
      if (sc.goal_static >= 0 && sc.goal_static < sc.n_static) {
        const int b = sc.goal_static;
        const float top = sc.st_center[b][2] + sc.st_half[b][2];
        goal = fabsf(ob.p.x - sc.st_center[b][0]) <= sc.st_half[b][0] && fabsf(ob.p.y - sc.st_center[b][1]) <= sc.st_half[b][1] &&
               ob.p.z >= top && ob.p.z <= top + 2.0f * sc.obj_half[2] && rest;
      } else if (sc.goal_static < 0) {
        goal = fabsf(ob.p.x - sc.goal_box_center[0]) <= sc.goal_box_half[0] &&
               fabsf(ob.p.y - sc.goal_box_center[1]) <= sc.goal_box_half[1] &&
               fabsf(ob.p.z - sc.goal_box_center[2]) <= sc.goal_box_half[2] && rest;
      }
      const float pose[7] = {ob.p.x, ob.p.y, ob.p.z, ob.q.w, ob.q.x, ob.q.y, ob.q.z};
      bool fin = !diverged;
#pragma unroll
      for (int i = 0; i < 7; ++i) fin = fin && isfinite(pose[i]);
      for (int j = 0; j < NJ; ++j) fin = fin && isfinite(L.at(R_Q + j)) && fabsf(L.at(R_Q + j)) < 1e3f;
      fin = fin && fabsf(ob.p.x) < 1e3f && fabsf(ob.p.y) < 1e3f && fabsf(ob.p.z) < 1e3f;
      const bool all_ok = ok_bits == (1u << n_act) - 1u;
      const int tier = !fin ? 3 : (all_ok ? (goal ? 0 : 1) : 2);
      EnvOut out;
      out.cost = fin ? sc.time_weight * dt * (float)unsuccessful : __int_as_float(0x7F800000);
      out.tier = tier;
      out.steps = steps;
#pragma unroll
      for (int i = 0; i < 7; ++i) out.pose[i] = pose[i];
      finish(out, row);
      total += steps;
    }
    // the next rollout for every lane whose rollout ended
    const bool need = live && ended;
    claim(need, row, live);
    if (need && live) {
      init_plan(row);
      diverged = false;
      steps = sc.horizon;
      calm = 0;
      t = 0;
    }
  }
  return total;
}


}  // namespace
}  // namespace cem
